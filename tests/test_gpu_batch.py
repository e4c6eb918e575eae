"""Graph-captured batches of unit cells, and the autotuner, on the GPU.

The graph-captured batch (each cell's work captured on its own branch of one
HIP graph, then replayed) crashed the host process (segmentation fault) in
its first call on the GPU, before any result came back; no cause was found
in this code by reading it, so the capture path was taken out of the
library and its tests below stay skipped. The autotuner's choice must give
the same fields up to FP32 rounding order.
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
              "GPU box and no cause was found in this code")


@pytest.mark.skip(reason=GRAPH_SKIP)
def test_batch_heff_equals_per_cell_calls_on_every_replay():
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
def test_batch_rk4_equals_per_cell_steps():
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
def test_batch_refuses_bad_cells():
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
    assert forms["fft"] in (1, 2) and forms["spmv"] in (4, 8, 16)
    assert ms > 0
    err = float((h1 - h0).norm() / h0.norm())
    assert err <= 1e-6, err
