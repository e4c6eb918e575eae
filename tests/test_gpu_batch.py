"""Batches of unit cells, and the autotuner, on the GPU.

A batch evaluates all its cells with one launch per stage (block-diagonal
local operators, multi-cell grid kernels). Per cell the arithmetic is that of
a single-cell evaluation with the same kernel forms and SpMV lanes, so the
packed results must equal the per-cell calls bit for bit, for H_eff and for
RK4 steps, on cells of every periodicity, two materials, uneven sizes and
every FFT form (whole planes, per-axis radix 2, mixed radix 2, 3, 5, 7); two
cells are also checked against the FP64 oracle.

An earlier graph-captured batch (each cell's work captured on its own branch
of one HIP graph, then replayed) crashed the host process (segmentation
fault) in its first call on the GPU, before any result came back; no cause
was found in this code by reading it, so that path was taken out of the
library and its tests (test_graph_batch_*) stay skipped; a batch's RK4 step
captured as one graph on a single stream with its second stream forked and
joined is tested in test_gpu_graph.py. The autotuner's
choice must give the same fields up to FP32 rounding order.
"""
import numpy as np
import pytest

from oracle import model
from paper_2409_13958_amd import meshgen as mg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
B = pytest.importorskip("paper_2409_13958_amd.binding")


def cells():
    probs = [mg.film_c1(),
             mg.kuhn_box((5, 7, 6), 1e-9, periodic=0b111, jitter=0.2, grid=(16, 16, 16)),
             mg.wire_c2(R=3e-9, period=6e-9, spacing=1.0e-9, n_layers=6, grid=(8, 8, 16)),
             mg.kuhn_box((6, 6, 6), 1e-9, periodic=0b111, jitter=0.2, Ms=[8e5, 3e5],
                         Aex=[1.3e-11, 0.7e-11], region_of=mg.ball_regions((6, 6, 6), 2.2),
                         grid=(16, 16, 16))]
    probs += mg.films_c4(4, nodes=(2e3, 6e3), period=(20e-9, 40e-9))
    out = []
    for p in probs:
        ctx = B.Context.from_problem(p, device=0)
        n, uon, nou, _ = ctx.query()
        out.append((p, ctx, nou))
    return out


GRAPH_SKIP = ("graph-captured batch removed: its first call crashed the host process on the "
              "GPU and no cause was found in this code")


@pytest.mark.skip(reason=GRAPH_SKIP)
def test_graph_batch_heff_equals_per_cell_calls_on_every_replay():
    cs = cells()
    print(f"[gpu batch] {len(cs)} cells, N' = {[c.n for _, c, _ in cs]}", flush=True)
    batch = B.Batch([c for _, c, _ in cs])
    ms = [torch.tensor(p.m[nou], dtype=torch.float32, device="cuda") for p, _, nou in cs]
    hs = [torch.empty_like(m) for m in ms]
    for rep in range(3):
        if rep:
            # new inputs in place (the graph reads through the same pointers)
            for m in ms:
                m.copy_(torch.roll(m, shifts=rep, dims=0))
        batch.heff(ms, hs)
        ref = []
        for (_, ctx, _), m in zip(cs, ms):
            h = torch.empty_like(m)
            ctx.heff(m, h)                      # eager work between replays
            ref.append(h)
        torch.cuda.synchronize()
        for k, (h, r) in enumerate(zip(hs, ref)):
            assert torch.equal(h, r), (rep, k)
    # one cell against the oracle (the same mesh as the film parity test)
    p, ctx, nou = cs[0]
    orc = model.Oracle(p)
    m0 = orc.unknown_values(p.m)
    ms[0].copy_(torch.tensor(p.m[nou], dtype=torch.float32))
    batch.heff(ms, hs)
    torch.cuda.synchronize()
    ref = orc.heff(m0, method="aim")[orc.uk[nou]]
    got = hs[0].cpu().numpy().astype(np.float64)
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(f"[gpu batch] film cell vs oracle: rel L2 {err:.2e}", flush=True)
    assert err <= 1e-5
    batch.close()


@pytest.mark.skip(reason=GRAPH_SKIP)
def test_graph_batch_rk4_equals_per_cell_steps():
    cs = cells()
    batch = B.Batch([c for _, c, _ in cs])
    mb = [torch.tensor(p.m[nou], dtype=torch.float64, device="cuda") for p, _, nou in cs]
    me = [m.clone() for m in mb]
    batch.llg_step(mb, 1e-13, 0.5, 3)
    batch.llg_step(mb, 1e-13, 0.5, 2)          # replay of the same graph
    for (_, ctx, _), m in zip(cs, me):
        ctx.llg_step(m, 1e-13, 0.5, 5)
    torch.cuda.synchronize()
    for k, (a, b) in enumerate(zip(mb, me)):
        assert torch.equal(a, b), k
        assert float((a.norm(dim=1) - 1).abs().max()) < 1e-13
    batch.close()


@pytest.mark.skip(reason=GRAPH_SKIP)
def test_graph_batch_refuses_bad_cells():
    p = mg.film_c1()
    ctx = B.Context.from_problem(p, device=0)
    with pytest.raises(B.PmfemError) as e:
        B.Batch([ctx, ctx])
    assert e.value.code == B.Status.EINVAL
    host = B.Context(device=-1)
    with pytest.raises(B.PmfemError) as e:
        B.Batch([ctx, host])
    assert e.value.code == B.Status.ESTATE


def test_autotune_keeps_the_fields():
    p = mg.kuhn_box((5, 7, 6), 1e-9, periodic=0b111, jitter=0.2, grid=(16, 16, 16))
    ctx = B.Context.from_problem(p, device=0)
    n, uon, nou, _ = ctx.query()
    m = torch.tensor(p.m[nou], dtype=torch.float32, device="cuda")
    h0, h1 = torch.empty_like(m), torch.empty_like(m)
    ctx.heff(m, h0)
    forms, ms = ctx.autotune(trials=5)
    ctx.heff(m, h1)
    torch.cuda.synchronize()
    print(f"[gpu batch] autotune: {forms}, {ms:.4f} ms per evaluation", flush=True)
    assert forms["anterp"] in (1, 2, 3) and forms["interp"] in (1, 2)
    assert forms["fft"] in (1, 2) and forms["spmv"] in (0, 4, 8, 16)
    assert ms > 0
    err = float((h1 - h0).norm() / h0.norm())
    assert err <= 1e-6, err


BATCH_FORMS = dict(anterp=3, interp=2, fft=2, spmv=4)


def batch_cells():
    probs = [mg.film_c1(),
             mg.kuhn_box((5, 7, 6), 1e-9, periodic=0b111, jitter=0.2, grid=(16, 16, 16)),
             mg.wire_c2(R=3e-9, period=6e-9, spacing=1.0e-9, n_layers=6, grid=(8, 8, 16)),
             mg.kuhn_box((6, 6, 6), 1e-9, periodic=0b111, jitter=0.2, Ms=[8e5, 3e5],
                         Aex=[1.3e-11, 0.7e-11], region_of=mg.ball_regions((6, 6, 6), 2.2),
                         grid=(16, 16, 16)),
             mg.kuhn_box((6, 6, 4), 1e-9, periodic=0b011, jitter=0.2, Ms=[8e5, 1.4e6],
                         Aex=[1.3e-11, 2e-11], region_of=lambda c: (c[:, 2] >= 2).astype(np.int32),
                         grid=(16, 16, 8))]
    probs += mg.films_c4(4, nodes=(2e3, 6e3), period=(20e-9, 40e-9))
    # a 256 x 256 plane does not fit in LDS: this cell takes the per-axis FFT
    # passes inside the batch
    probs.append(mg.kuhn_box((4, 4, 1), 2e-9, periodic=0b011, jitter=0.1, grid=(256, 256, 4)))
    # extents with factors 3, 5 and 7: the mixed-radix passes inside the batch
    # (the films above have such extents too)
    probs.append(mg.kuhn_box((6, 5, 2), 1e-9, periodic=0b011, jitter=0.2, grid=(12, 20, 6)))
    probs.append(mg.kuhn_box((5, 6, 5), 1e-9, periodic=0b111, jitter=0.2, grid=(15, 14, 21)))
    out = []
    for p in probs:
        ctx = B.Context.from_problem(p, device=0)
        for stage, v in BATCH_FORMS.items():
            try:
                ctx.set_variant(stage, v)
            except B.PmfemError:
                ctx.set_variant(stage, 1)     # the form the batch takes when this one does not fit
        n, uon, nou, _ = ctx.query()
        out.append((p, ctx, nou))
    return out


def test_batch_heff_equals_per_cell_calls():
    cs = batch_cells()
    batch = B.Batch([c for _, c, _ in cs], spmv_lanes=4)
    off = batch.offsets
    print(f"[gpu batch] {len(cs)} cells, N' = {np.diff(off).tolist()}", flush=True)
    m = torch.cat([torch.tensor(p.m[nou], dtype=torch.float32) for p, _, nou in cs]).cuda()
    h, h2 = torch.empty_like(m), torch.empty_like(m)
    batch.heff(m, h)
    batch.heff(m, h2)
    hms = torch.empty_like(m)
    batch.heff(m, hms, terms=B.TERM_MS)
    ref, ref_ms = [], []
    for k, (p, ctx, nou) in enumerate(cs):
        mk = m[off[k]:off[k + 1]].contiguous()
        r, rm = torch.empty_like(mk), torch.empty_like(mk)
        ctx.heff(mk, r)
        ctx.heff(mk, rm, terms=B.TERM_MS)
        ref.append(r)
        ref_ms.append(rm)
    torch.cuda.synchronize()
    assert torch.equal(h, h2)
    for k in range(len(cs)):
        assert torch.equal(h[off[k]:off[k + 1]], ref[k]), k
        assert torch.equal(hms[off[k]:off[k + 1]], ref_ms[k]), k
    # three cells against the FP64 oracle, the last a mixed-radix one
    for k in (0, 3, len(cs) - 1):
        p, ctx, nou = cs[k]
        orc = model.Oracle(p)
        r = orc.heff(orc.unknown_values(p.m), method="aim")[orc.uk[nou]]
        got = h[off[k]:off[k + 1]].cpu().numpy().astype(np.float64)
        err = float(np.linalg.norm(got - r) / np.linalg.norm(r))
        print(f"[gpu batch] cell {k} vs oracle: rel L2 {err:.2e}", flush=True)
        assert err <= 1e-5
    batch.close()


def test_batch_rk4_equals_per_cell_steps():
    cs = batch_cells()
    batch = B.Batch([c for _, c, _ in cs], spmv_lanes=4)
    off = batch.offsets
    m = torch.cat([torch.tensor(p.m[nou], dtype=torch.float64) for p, _, nou in cs]).cuda()
    me = [m[off[k]:off[k + 1]].clone() for k in range(len(cs))]
    batch.llg_step(m, 1e-13, 0.5, 3)
    for (_, ctx, _), mk in zip(cs, me):
        ctx.llg_step(mk, 1e-13, 0.5, 3)
    torch.cuda.synchronize()
    for k in range(len(cs)):
        assert torch.equal(m[off[k]:off[k + 1]], me[k]), k
    assert float((m.norm(dim=1) - 1).abs().max()) < 1e-13
    batch.close()


def test_batch_refuses_unfit_cells():
    p = mg.film_c1()
    a = B.Context.from_problem(p, device=0)
    with pytest.raises(B.PmfemError) as e:
        B.Batch([a, a])
    assert e.value.code == B.Status.EINVAL
    other = B.Context.from_problem(mg.kuhn_box((6, 6, 2), 1e-9, periodic=0b011, jitter=0.2,
                                               grid=(16, 16, 4)), device=0, order_p=2,
                                   near_boxes=1)
    with pytest.raises(B.PmfemError) as e:
        B.Batch([a, other])
    assert e.value.code == B.Status.EINVAL
    assert "order" in str(e.value)
    host = B.Context(device=-1)
    with pytest.raises(B.PmfemError) as e:
        B.Batch([a, host])
    assert e.value.code == B.Status.ESTATE
