"""GPU (gfx950) effective field through the C ABI against the FP64 oracle.

Bar (FP32 path vs the FP64 oracle running the same AIM): relative L2 error
<= 1e-5 per field (H_ex, H_ms, H_eff), on every mesh here; grid convolution
alone <= 1e-6; repeated calls bitwise identical (no atomics anywhere).
"""
import numpy as np
import pytest

from oracle import model
from paper_2409_13958_amd import meshgen as mg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
B = pytest.importorskip("paper_2409_13958_amd.binding")

TOL = 1e-5


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# kernel forms: staged line anterpolation, the basic forms of each stage and
# scatter anterpolation (the default choice)
FORMS = {"staged": dict(anterp=2, interp=2, fft=2, spmv=8),
         "basic": dict(anterp=1, interp=1, fft=1, spmv=16),
         "scatter": dict(anterp=3, spmv=4)}


def lib_fields(prob, m_nodes, forms=None, **kw):
    ctx = B.Context.from_problem(prob, device=0, **kw)
    for stage, v in (forms or {}).items():
        ctx.set_variant(stage, v)
    n, uon, nou, _ = ctx.query()
    m = torch.tensor(np.asarray(m_nodes)[nou], dtype=torch.float32, device="cuda")
    h = torch.empty_like(m)
    hex_ = torch.empty_like(m)
    q = torch.empty(n, dtype=torch.float32, device="cuda")
    u = torch.empty_like(q)
    hms = torch.empty_like(m)
    ctx.heff_parts(m, h, q, u, hex_)
    ctx.heff(m, hms, terms=B.TERM_MS)
    torch.cuda.synchronize()
    return ctx, nou, {k: v.cpu().numpy().astype(np.float64)
                      for k, v in dict(h=h, hex=hex_, hms=hms, q=q, u=u).items()}


SMALL = {
    "film_c1": lambda: mg.film_c1(),
    "box3d_jitter_ragged": lambda: mg.kuhn_box((5, 7, 6), 1e-9, periodic=0b111, jitter=0.2,
                                               grid=(16, 16, 16)),
    "wire_small": lambda: mg.wire_c2(R=3e-9, period=6e-9, spacing=1.0e-9, n_layers=6,
                                     grid=(8, 8, 16)),
    "film_xz": lambda: mg.kuhn_box((6, 3, 6), 1e-9, periodic=0b101, jitter=0.15, grid=(16, 4, 16)),
    "film_long_axis_512": lambda: mg.kuhn_box((40, 4, 1), 2e-9, periodic=0b011, grid=(512, 16, 4)),
    "order5_radius3": lambda: mg.kuhn_box((6, 6, 2), 1e-9, periodic=0b011, jitter=0.2,
                                          grid=(32, 32, 8)),
    # the remaining Lagrange orders and near radii, and a cell with no
    # periodic axis (every FFT axis zero-padded)
    "open_box_p1_rb0": lambda: mg.kuhn_box((5, 5, 4), 1e-9, periodic=0, jitter=0.2,
                                           grid=(8, 8, 8)),
    "film_p2_rb1": lambda: mg.kuhn_box((6, 6, 2), 1e-9, periodic=0b011, jitter=0.2,
                                       grid=(16, 16, 4)),
    "slab_p4_rb1": lambda: mg.kuhn_box((5, 6, 4), 1e-9, periodic=0b011, jitter=0.2,
                                       grid=(16, 16, 8)),
    # p = 4 on 16 periodic points: the preferred z tiles (5 boxes) leave a
    # short last tile, so the scatter plan takes tiles that divide the axis
    "box3d_p4_rb1": lambda: mg.kuhn_box((5, 6, 5), 1e-9, periodic=0b111, jitter=0.2,
                                        grid=(16, 16, 16)),
    # two materials (Sec. 3.2.1: faces between materials of different Ms
    # carry surface charge): a ball of another Ms and A inside a jittered
    # 3D-periodic cell, and a bilayer film (interface plus outer faces)
    "inclusion_3d": lambda: mg.kuhn_box((6, 6, 6), 1e-9, periodic=0b111, jitter=0.2,
                                        Ms=[8e5, 3e5], Aex=[1.3e-11, 0.7e-11],
                                        region_of=mg.ball_regions((6, 6, 6), 2.2),
                                        grid=(16, 16, 16)),
    "bilayer_film": lambda: mg.kuhn_box((6, 6, 4), 1e-9, periodic=0b011, jitter=0.2,
                                        Ms=[8e5, 1.4e6], Aex=[1.3e-11, 2e-11],
                                        region_of=lambda c: (c[:, 2] >= 2).astype(np.int32),
                                        grid=(16, 16, 8)),
}
KW = {"order5_radius3": dict(order_p=5, near_boxes=3),
      "open_box_p1_rb0": dict(order_p=1, near_boxes=0),
      "film_p2_rb1": dict(order_p=2, near_boxes=1),
      "slab_p4_rb1": dict(order_p=4, near_boxes=1),
      "box3d_p4_rb1": dict(order_p=4, near_boxes=1)}


@pytest.mark.parametrize("name", sorted(SMALL))
def test_heff_parity_small(name):
    prob = SMALL[name]()
    kw = KW.get(name, {})
    print(f"[gpu parity] {name} nodes={prob.n_nodes}", flush=True)
    orc = model.Oracle(prob, order_p=kw.get("order_p"), near_boxes=kw.get("near_boxes"))
    m = orc.unknown_values(prob.m)
    ref = dict(h=orc.heff(m, method="aim"), hex=orc.heff(m, method="aim", terms=("ex",)),
               hms=orc.heff(m, method="aim", terms=("ms",)), q=orc.charges(m),
               u=orc.potential(m, None, "aim"))
    for form, forms in FORMS.items():
        print(f"[gpu parity] {name} forms={form}", flush=True)
        ctx, nou, got = lib_fields(prob, prob.m, forms, **kw)
        perm = orc.uk[nou]
        errs = {k: rel(got[k], r[perm]) for k, r in ref.items()}
        print(f"[gpu parity] {name} {form} rel L2: "
              + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
        for k, v in errs.items():
            assert v <= TOL, (form, k, v)


@pytest.mark.parametrize("fft", [1, 2])
@pytest.mark.parametrize("case", ["wire_small", "box3d_jitter_ragged"])
def test_grid_convolution_alone(case, fft):
    prob = SMALL[case]()
    ctx = B.Context.from_problem(prob, device=0)
    ctx.set_variant("fft", fft)
    orc = model.Oracle(prob)
    N = orc.aim.grid.N
    rng = np.random.default_rng(3)
    Q = rng.standard_normal(tuple(N))
    qg = torch.tensor(Q.transpose(2, 1, 0).copy(), dtype=torch.float32, device="cuda")
    ug = torch.empty_like(qg)
    ctx.grid_convolve(qg, ug)
    U = ug.cpu().numpy().astype(np.float64).transpose(2, 1, 0)
    ref = orc.aim.convolve(Q) / (4 * np.pi)
    err = rel(U, ref)
    print(f"[gpu parity] convolution {case} fft={fft}: rel L2 {err:.2e}", flush=True)
    assert err <= 1e-6


def test_bitwise_deterministic_and_terms():
    prob = SMALL["box3d_jitter_ragged"]()
    ctx = B.Context.from_problem(prob, device=0)
    n, uon, nou, _ = ctx.query()
    m = torch.tensor(prob.m[nou], dtype=torch.float32, device="cuda")
    h1, h2, hex_, hms = (torch.empty_like(m) for _ in range(4))
    ctx.heff(m, h1)
    ctx.heff(m, h2)
    ctx.heff(m, hex_, terms=B.TERM_EX)
    ctx.heff(m, hms, terms=B.TERM_MS, h_applied=[1e4, -2e4, 3e4])
    torch.cuda.synchronize()
    assert torch.equal(h1, h2)
    ha = torch.tensor([1e4, -2e4, 3e4], dtype=torch.float32, device="cuda")
    assert torch.allclose(hex_ + hms - ha, h1, rtol=1e-6, atol=1e-6 * float(h1.abs().max()))
    # uniform magnetisation, along an axis or not: exactly no exchange field
    # (the kernel sums L_nk (m_k - m_n))
    for d in ([0.0, 0.0, 1.0], [0.48, 0.6, 0.64]):
        mu = torch.tensor(d, dtype=torch.float32, device="cuda").expand_as(m).contiguous()
        ctx.heff(mu, hex_, terms=B.TERM_EX)
        torch.cuda.synchronize()
        assert float(hex_.abs().max()) == 0.0


def test_exchange_of_a_nearly_uniform_state():
    """m = uniform + 1e-3 random, renormalised: the exchange field is 1e-3 of
    its scale for a random m, and the rounding of the FP32 row sums alone
    (about 6e-8 of the diagonal per entry) would be 1e-4 of it; the
    difference form keeps the FP32 result within the bar of the oracle."""
    prob = SMALL["box3d_jitter_ragged"]()
    orc = model.Oracle(prob, with_aim=False)
    rng = np.random.Generator(np.random.PCG64(11))
    mn = np.array([0.48, 0.6, 0.64]) + 1e-3 * rng.standard_normal((prob.n_nodes, 3))
    mn /= np.linalg.norm(mn, axis=1, keepdims=True)
    ctx = B.Context.from_problem(prob, device=0)
    n, uon, nou, _ = ctx.query()
    mo = orc.unknown_values(mn)
    perm = orc.uk[nou]
    # both sides take the same value per unknown
    m = torch.tensor(mo[perm], dtype=torch.float32, device="cuda")
    hex_ = torch.empty_like(m)
    ctx.heff(m, hex_, terms=B.TERM_EX)
    torch.cuda.synchronize()
    ref = orc.ops.exchange(m.cpu().numpy().astype(np.float64)[np.argsort(perm)])
    err = rel(hex_.cpu().numpy().astype(np.float64), ref[perm])
    print(f"[gpu parity] exchange of a nearly uniform m: rel L2 {err:.2e}", flush=True)
    assert err <= TOL


def test_energy_matches_oracle():
    prob = mg.film_c1()
    ctx = B.Context.from_problem(prob, device=0)
    n, uon, nou, _ = ctx.query()
    orc = model.Oracle(prob)
    m = orc.unknown_values(prob.m)
    e_ex, e_ms, _ = orc.energy(m)
    m64 = torch.tensor(prob.m[nou], dtype=torch.float64, device="cuda")
    g_ex, g_ms = ctx.energy(m64)
    assert g_ex == pytest.approx(e_ex, rel=1e-5)
    assert g_ms == pytest.approx(e_ms, rel=1e-5)


def test_macrospin_llg_closed_form():
    p = mg.kuhn_box((3, 3, 3), 2e-9, periodic=0b111, Ms=8e5, grid=(16, 16, 16))
    ctx = B.Context.from_problem(p, device=0)
    n = ctx.n
    th0, ph0, Hap, alpha = 0.9, 0.3, 2e5, 0.3
    m0 = np.array([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)])
    m = torch.tensor(np.tile(m0, (n, 1)), dtype=torch.float64, device="cuda")
    dt, steps = 5e-14, 80
    ctx.llg_step(m, dt, alpha, steps, h_applied=[0.0, 0.0, Hap])
    torch.cuda.synchronize()
    g = model.GAMMA0 * Hap / (1 + alpha ** 2)
    t = dt * steps
    th = 2 * np.arctan(np.tan(th0 / 2) * np.exp(-alpha * g * t))
    ph = ph0 + g * t
    ex = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    got = m.cpu().numpy()
    assert np.abs(got - ex[None, :]).max() < 1e-5
    assert np.allclose(np.linalg.norm(got, axis=1), 1.0, atol=1e-13)


def test_film_llg_trajectory_against_oracle():
    """100 RK4 steps of 0.1 ps, alpha = 0.5, exchange + magnetostatic field."""
    prob = mg.film_c1()
    ctx = B.Context.from_problem(prob, device=0)
    n, uon, nou, _ = ctx.query()
    orc = model.Oracle(prob)
    perm = orc.uk[nou]
    m0 = orc.unknown_values(prob.m)
    ref = orc.rk4(m0, 1e-13, 0.5, 100, method="aim")[perm]
    m = torch.tensor(prob.m[nou], dtype=torch.float64, device="cuda")
    ctx.llg_step(m, 1e-13, 0.5, 100)
    torch.cuda.synchronize()
    got = m.cpu().numpy()
    err = rel(got, ref)
    print(f"[gpu parity] film 100-step trajectory rel L2 = {err:.3e}")
    # FP32 fields in an FP64 trajectory: about 5e-8 measured
    assert err < 1e-6
    assert np.allclose(np.linalg.norm(got, axis=1), 1.0, atol=1e-13)


# FFT extents that are products of 2, 3, 5 and 7 but not powers of two take
# the mixed-radix per-axis passes (the plane form needs powers of two)
MIXED = {
    "film_12x20x6": lambda: mg.kuhn_box((6, 5, 2), 1e-9, periodic=0b011, jitter=0.2,
                                        grid=(12, 20, 6)),
    "box3d_15x14x21": lambda: mg.kuhn_box((5, 6, 5), 1e-9, periodic=0b111, jitter=0.2,
                                          grid=(15, 14, 21)),
}


@pytest.mark.parametrize("name", sorted(MIXED))
def test_heff_parity_mixed_radix(name):
    prob = MIXED[name]()
    print(f"[gpu parity] {name} nodes={prob.n_nodes}", flush=True)
    orc = model.Oracle(prob)
    m = orc.unknown_values(prob.m)
    ref = dict(h=orc.heff(m, method="aim"), hms=orc.heff(m, method="aim", terms=("ms",)),
               u=orc.potential(m, None, "aim"))
    tried = 0
    for anterp, fft in ((0, 0), (1, 1), (2, 2), (3, 1)):
        ctx = B.Context.from_problem(prob, device=0)
        try:
            ctx.set_variant("anterp", anterp)
        except B.PmfemError:
            continue                     # this form's plan does not fit the grid
        ctx.set_variant("fft", fft)
        tried += 1
        n, uon, nou, _ = ctx.query()
        mt = torch.tensor(prob.m[nou], dtype=torch.float32, device="cuda")
        h, hms, u = torch.empty_like(mt), torch.empty_like(mt), torch.empty(n, device="cuda")
        ctx.heff_parts(mt, h, None, u, None)
        ctx.heff(mt, hms, terms=B.TERM_MS)
        torch.cuda.synchronize()
        perm = orc.uk[nou]
        got = dict(h=h, hms=hms, u=u)
        errs = {k: rel(got[k].cpu().numpy().astype(np.float64), r[perm]) for k, r in ref.items()}
        print(f"[gpu parity] {name} anterp={anterp} fft={fft} rel L2: "
              + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
        for k, v in errs.items():
            assert v <= TOL, (anterp, k, v)
    assert tried >= 2


@pytest.mark.parametrize("case", sorted(MIXED))
def test_grid_convolution_mixed_radix(case):
    """Both forms of the mixed-radix passes: whole planes in LDS for x and y
    (fft 2) and one axis per pass (fft 1)."""
    prob = MIXED[case]()
    orc = model.Oracle(prob)
    N = orc.aim.grid.N
    Q = np.random.default_rng(5).standard_normal(tuple(N))
    ref = orc.aim.convolve(Q) / (4 * np.pi)
    for fft in (2, 1):
        ctx = B.Context.from_problem(prob, device=0)
        ctx.set_variant("fft", fft)
        qg = torch.tensor(Q.transpose(2, 1, 0).copy(), dtype=torch.float32, device="cuda")
        ug = torch.empty_like(qg)
        ctx.grid_convolve(qg, ug)
        U = ug.cpu().numpy().astype(np.float64).transpose(2, 1, 0)
        err = rel(U, ref)
        print(f"[gpu parity] convolution {case} (mixed radix, fft={fft}): rel L2 {err:.2e}",
              flush=True)
        assert err <= 1e-6


def test_grid_convolution_surrogate_workload_size():
    """The grid of the surrogate workload, a film of 512 x 512 x 16 grid
    points (FFT extents 512 x 512 x 32): a 512 x 512 plane does not fit in
    LDS, so the convolution takes the per-axis radix-2 passes at their
    longest lines; against the oracle's FFT convolution with its own PGF."""
    prob = mg.kuhn_box((16, 16, 2), 32e-9, periodic=0b011, jitter=0.1, grid=(512, 512, 16))
    orc = model.Oracle(prob)
    N = orc.aim.grid.N
    Q = np.random.default_rng(7).standard_normal(tuple(N))
    ref = orc.aim.convolve(Q) / (4 * np.pi)
    ctx = B.Context.from_problem(prob, device=0)
    with pytest.raises(B.PmfemError):
        ctx.set_variant("fft", 2)        # the plane form does not fit this grid
    qg = torch.tensor(Q.transpose(2, 1, 0).copy(), dtype=torch.float32, device="cuda")
    ug = torch.empty_like(qg)
    ctx.grid_convolve(qg, ug)
    U = ug.cpu().numpy().astype(np.float64).transpose(2, 1, 0)
    err = rel(U, ref)
    errmax = float(np.abs(U - ref).max() / np.abs(ref).max())
    print(f"[gpu parity] convolution 512x512x16 film: rel L2 {err:.2e}, max {errmax:.2e}",
          flush=True)
    assert err <= 1e-6 and errmax <= 1e-5
