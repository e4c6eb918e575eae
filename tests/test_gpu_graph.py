"""RK4 steps replayed from a captured HIP graph (pmfem_llg_step_graph).

One RK4 step of a single context (its kernels and their fork to the second
stream and back) is captured once and launched per step; the results must be
those of the eager pmfem_llg_step bit for bit, on every replay, with the
program's own eager work and synchronisations between the replays, and after
a new capture when the step's arguments change.
"""
import numpy as np
import pytest

from paper_2409_13958_amd import meshgen as mg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
B = pytest.importorskip("paper_2409_13958_amd.binding")


def test_graph_steps_equal_eager_steps_on_every_replay():
    prob = mg.film_c1()
    ctx = B.Context.from_problem(prob, device=0)
    n, uon, nou, _ = ctx.query()
    m0 = torch.tensor(prob.m[nou], dtype=torch.float64, device="cuda")
    me, mg_ = m0.clone(), m0.clone()
    h = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    for rep in range(4):
        ctx.llg_step(me, 1e-13, 0.5, 2)
        ctx.llg_step_graph(mg_, 1e-13, 0.5, 2)
        ctx.heff(me.float().contiguous(), h)        # eager work between the replays
        torch.cuda.synchronize()
        assert torch.equal(me, mg_), rep
    # other arguments: a new capture (time step, damping, applied field)
    for dt, alpha, ha in ((2e-13, 0.5, None), (2e-13, 0.1, [1e4, 0.0, -2e4]),
                          (2e-13, 0.1, [1e4, 0.0, -2e4])):
        ctx.llg_step(me, dt, alpha, 3, h_applied=ha)
        ctx.llg_step_graph(mg_, dt, alpha, 3, h_applied=ha)
        torch.cuda.synchronize()
        assert torch.equal(me, mg_), (dt, alpha, ha)
    # another magnetisation buffer: captured anew for it
    m2e, m2g = m0.clone(), m0.clone()
    ctx.llg_step(m2e, 1e-13, 0.5, 2)
    ctx.llg_step_graph(m2g, 1e-13, 0.5, 2)
    torch.cuda.synchronize()
    assert torch.equal(m2e, m2g)
    assert float((mg_.norm(dim=1) - 1).abs().max()) < 1e-13


def test_graph_step_refuses_bad_arguments():
    ctx = B.Context.from_problem(mg.film_c1(), device=0)
    m = torch.zeros((ctx.n, 3), dtype=torch.float64, device="cuda")
    m[:, 2] = 1.0
    for dt, alpha, n in ((-1e-13, 0.5, 1), (1e-13, -0.1, 1), (1e-13, 0.5, -1)):
        with pytest.raises(B.PmfemError) as e:
            ctx.llg_step_graph(m, dt, alpha, n)
        assert e.value.code == B.Status.EINVAL


def test_batch_graph_steps_equal_eager_batch_steps():
    """The batch's RK4 step captured as one graph (all cells, one launch per
    stage, the second stream forked and joined): every replay equals the
    eager batch steps bit for bit, with eager work between the replays."""
    probs = [mg.film_c1(),
             mg.kuhn_box((5, 7, 6), 1e-9, periodic=0b111, jitter=0.2, grid=(16, 16, 16)),
             mg.kuhn_box((5, 6, 5), 1e-9, periodic=0b111, jitter=0.2, grid=(15, 14, 21))]
    probs += mg.films_c4(3, nodes=(2e3, 6e3), period=(20e-9, 40e-9))
    ctxs = [B.Context.from_problem(p, device=0) for p in probs]
    noun = [c.query()[2] for c in ctxs]
    batch = B.Batch(ctxs)
    m0 = torch.cat([torch.tensor(p.m[nou], dtype=torch.float64) for p, nou in zip(probs, noun)]
                   ).cuda()
    me, mg_ = m0.clone(), m0.clone()
    h = torch.empty(me.shape, dtype=torch.float32, device="cuda")
    for rep in range(3):
        batch.llg_step(me, 1e-13, 0.5, 2)
        batch.llg_step_graph(mg_, 1e-13, 0.5, 2)
        batch.heff(me.float().contiguous(), h)      # eager work between the replays
        torch.cuda.synchronize()
        assert torch.equal(me, mg_), rep
    batch.llg_step(me, 3e-13, 0.2, 2)
    batch.llg_step_graph(mg_, 3e-13, 0.2, 2)        # new arguments: captured anew
    torch.cuda.synchronize()
    assert torch.equal(me, mg_)
    batch.close()
