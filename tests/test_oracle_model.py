"""Physics pins of the oracle's assembled H_eff and LLG (paper Eqs. heff, hms, llg).

* A uniformly magnetised 2D-periodic film has H_ms = -Ms n (out of plane) and
  0 (in plane). The nodal point-charge model is exact only in the limit of
  an exact-integration radius covering the cell, so the out-of-plane case is
  checked as a convergence in the radius kappa.
* An axially magnetised 1D-periodic wire with vertical lateral faces has no
  charge at all, hence no demagnetising field.
* Macrospin: uniform m in a fully filled unjittered 3D-periodic cell feels
  only the applied field; RK4 follows the closed-form damped precession.
* Energy: H_ms = -(1/(mu0 mu_n)) dE_ms/dm_n for the symmetric direct
  operator; with alpha = 0 the exchange-only dynamics conserves energy.
"""
import numpy as np
import pytest

from oracle import model
from paper_2409_13958_amd import meshgen as mg

MS = 8e5


@pytest.fixture(scope="module")
def film():
    return mg.film_c1()


def test_film_out_of_plane_converges_to_minus_ms(film):
    errs = []
    for kappa in (1.0, 2.0):
        o = model.Oracle(film, z0_radius=kappa, with_aim=False)
        m = np.tile([0.0, 0.0, 1.0], (o.n, 1))
        H = o.heff(m, method="direct", terms=("ms",))
        assert np.abs(H[:, :2]).max() < 1e-9 * MS
        errs.append(np.abs(H[:, 2] / MS + 1).max())
    assert errs[0] < 0.05 and errs[1] < 0.01 and errs[1] < errs[0] / 4


def test_film_in_plane_has_no_field(film):
    o = model.Oracle(film, with_aim=False)
    m = np.tile([0.6, 0.8, 0.0], (o.n, 1))
    assert np.abs(o.charges(m)).max() < 1e-12 * MS * 4e-18
    H = o.heff(m, method="direct", terms=("ms",))
    assert np.abs(H).max() < 1e-9 * MS


def test_aim_matches_direct_on_film(film):
    o = model.Oracle(film)
    m = o.unknown_values(film.m)
    Ha = o.heff(m, method="aim", terms=("ms",))
    Hd = o.heff(m, method="direct", terms=("ms",))
    assert np.linalg.norm(Ha - Hd) / np.linalg.norm(Hd) < 1e-2


def test_rows_subset_matches_full(film):
    o = model.Oracle(film)
    m = o.unknown_values(film.m)
    rows = np.array([0, 17, 99, 150, 199])
    Hf = o.heff(m, method="aim")
    Hr = o.heff(m, rows=rows, method="aim")
    assert np.allclose(Hr, Hf[rows], rtol=1e-12, atol=1e-9)


def test_axial_wire_has_no_demag_field():
    w = mg.wire_c2(R=3e-9, period=6e-9, spacing=1.0e-9, n_layers=6, grid=(8, 8, 16))
    o = model.Oracle(w)
    m = np.tile([0.0, 0.0, 1.0], (o.n, 1))
    q = o.charges(m)
    assert np.abs(q).max() < 1e-12 * 1.4e6 * 1e-18
    H = o.heff(m, method="aim", terms=("ms",))
    assert np.abs(H).max() < 1e-9 * 1.4e6


def test_macrospin_precession_closed_form():
    # h = 2 nm keeps the exchange spectrum inside the RK4 stability region
    p = mg.kuhn_box((3, 3, 3), 2e-9, periodic=0b111, Ms=MS, grid=(12, 12, 12))
    o = model.Oracle(p)
    th0, ph0 = 0.9, 0.3
    m0 = np.tile([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)], (o.n, 1))
    Hap = 2e5
    alpha = 0.3
    H = o.heff(m0, method="aim")
    assert np.abs(H).max() < 1e-6 * MS
    dt, n = 5e-14, 80
    m = o.rk4(m0, dt, alpha, n, method="aim", h_app=[0.0, 0.0, Hap])
    t = dt * n
    g = model.GAMMA0 * Hap / (1 + alpha ** 2)
    th = 2 * np.arctan(np.tan(th0 / 2) * np.exp(-alpha * g * t))
    ph = ph0 + g * t
    ex = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    assert np.abs(m - ex[None, :]).max() < 1e-8
    assert np.allclose(np.linalg.norm(m, axis=1), 1.0, atol=1e-14)


def test_ms_energy_derivative_direct_without_correction():
    p = mg.kuhn_box((3, 3, 2), 1e-9, periodic=0b011, jitter=0.2, grid=(12, 12, 4))
    o = model.Oracle(p, with_aim=False)
    rng = np.random.default_rng(21)
    m = rng.standard_normal((o.n, 3))

    def e_ms(mm):
        q = o.charges(mm)
        return 0.5 * model.MU0 * q @ o.potential(mm, None, "direct", z0=False)
    H = o.ops.gradient_field(o.potential(m, None, "direct", z0=False))
    eps = 1e-4
    for n, c in [(0, 2), (7, 0), (o.n - 1, 1)]:
        mp, mm_ = m.copy(), m.copy()
        mp[n, c] += eps
        mm_[n, c] -= eps
        dE = (e_ms(mp) - e_ms(mm_)) / (2 * eps)
        assert H[n, c] == pytest.approx(-dE / (model.MU0 * o.ops.mu[n]), rel=1e-6)


def test_exchange_only_energy_conserved_without_damping():
    p = mg.kuhn_box((4, 4, 1), 2e-9, periodic=0b011, jitter=0.2, grid=(12, 12, 4))
    o = model.Oracle(p, with_aim=False)
    m0 = o.unknown_values(p.m)
    e0 = o.ops.exchange_energy(m0)
    m = o.rk4(m0, 2e-15, 0.0, 50, method="direct", terms=("ex",))
    e1 = o.ops.exchange_energy(m)
    assert abs(e1 - e0) < 1e-6 * abs(e0)
    # and with damping the energy decreases
    m = o.rk4(m0, 2e-15, 0.5, 50, method="direct", terms=("ex",))
    assert o.ops.exchange_energy(m) < e0


def test_aim_error_report_on_the_film(film):
    # the full-size AIM error script, run with every unknown of the film as a
    # sample, reports the whole-film AIM-vs-direct error of H_ms
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    o = model.Oracle(film)
    m = o.unknown_values(film.m)
    Ha = o.heff(m, method="aim", terms=("ms",))
    Hd = o.heff(m, method="direct", terms=("ms",))
    want = np.linalg.norm(Ha - Hd) / np.linalg.norm(Hd)
    out = subprocess.run([sys.executable, os.path.join(root, "oracle", "report_aim_error.py"),
                          "film_c1", str(o.n), "2"], capture_output=True, text=True, timeout=300,
                         check=True).stdout
    line = next(ln for ln in out.splitlines() if ln.startswith("H_ms at the samples rel L2"))
    assert float(line.split()[-1]) == pytest.approx(want, rel=1e-3)


# --- two materials: a 3D-periodic laminate (Sec. 3.2.1: surface charges on
# boundaries between materials of different saturation magnetisation) -------

LAM_M = (8e5, 3e5)
LAM_A = (1.3e-11, 0.7e-11)
LAM_NZ = 16


def laminate(m, jitter=0.0, grid=(12, 12, 48)):
    """4 x 4 x 16 Kuhn cells of 1 nm, periodic on all axes, region 0 for the
    lower 8 cell layers and region 1 for the upper 8 (two interfaces per
    period, at z = 0 and z = 8 nm)."""
    return mg.kuhn_box((4, 4, LAM_NZ), 1e-9, periodic=0b111, Ms=list(LAM_M), Aex=list(LAM_A),
                       region_of=lambda c: (c[:, 2] >= LAM_NZ // 2).astype(np.int32),
                       grid=grid, m=m, jitter=jitter, name="laminate")


def _layer_distance(o):
    zi = np.round(np.mod(o.pos[:, 2] / 1e-9, LAM_NZ)).astype(int)
    half = LAM_NZ // 2
    return zi, np.minimum(zi % half, half - zi % half)


def test_laminate_normal_magnetisation_closed_form():
    """m = z in both layers: B_z is uniform and the periodic potential gives
    int H_z dz = 0 over a period, so H_z = -(Ms_i - Mbar) in layer i, with
    Mbar the thickness-weighted mean. The point-charge lattice on each
    interface differs from the uniform sheet only by terms that decay like
    exp(-2 pi d / a) (a = 1 nm node spacing), so three layers away from an
    interface the closed form holds to 1e-5; next to it the element-exact
    correction carries the sheet (a few per cent at kappa = 1; counting the
    interface faces as interior leaves a 31 % error there)."""
    o = model.Oracle(laminate([0.0, 0.0, 1.0]))
    m = np.tile([0.0, 0.0, 1.0], (o.n, 1))
    q = o.charges(m)
    zi, d = _layer_distance(o)
    dm = LAM_M[0] - LAM_M[1]
    # rho = -div M: M_z rises by dM going up through z = 0 and falls by dM
    # through z = 8 nm, so the sheets carry -dM and +dM per unit area
    area = 16e-18
    assert np.sum(q[zi == 0]) == pytest.approx(-dm * area, rel=1e-12)
    assert np.sum(q[zi == LAM_NZ // 2]) == pytest.approx(dm * area, rel=1e-12)
    assert np.abs(q[d > 0]).max() < 1e-12 * dm * area
    mbar = 0.5 * (LAM_M[0] + LAM_M[1])
    ex = np.where(zi < LAM_NZ // 2, -(LAM_M[0] - mbar), -(LAM_M[1] - mbar))
    for method in ("direct", "aim"):
        H = o.heff(m, method=method, terms=("ms",))
        assert np.abs(H[:, :2]).max() < 1e-9 * LAM_M[0]
        err = np.abs(H[:, 2] - ex) / abs(LAM_M[0] - mbar)
        assert err[d >= 3].max() < 1e-5
        assert err[(d == 1) | (d == 2)].max() < 0.05


def test_laminate_in_plane_has_no_field():
    o = model.Oracle(laminate([0.6, 0.8, 0.0]), with_aim=False)
    m = np.tile([0.6, 0.8, 0.0], (o.n, 1))
    assert np.abs(o.charges(m)).max() < 1e-12 * LAM_M[0] * 1e-18
    H = o.heff(m, method="direct", terms=("ms",))
    assert np.abs(H).max() < 1e-9 * LAM_M[0]


def test_laminate_exchange_per_material():
    """m = (cos kx, sin kx, 0): on the unjittered Kuhn lattice the P1
    exchange is the 7-point Laplacian, so a node whose tetrahedra all lie in
    region i has H_ex = -(2 A_i / (mu0 Ms_i)) (2 / h^2)(1 - cos kh) m."""
    h, k = 1e-9, 2 * np.pi / 4e-9
    p = laminate(lambda xyz: np.stack([np.cos(k * xyz[:, 0]), np.sin(k * xyz[:, 0]),
                                       np.zeros(len(xyz))], axis=1))
    o = model.Oracle(p, with_aim=False)
    m = o.unknown_values(p.m)
    H = o.ops.exchange(m)
    zi, d = _layer_distance(o)
    for r in (0, 1):
        sel = (d >= 1) & ((zi < LAM_NZ // 2) == (r == 0))
        c = -(2 * LAM_A[r] / (model.MU0 * LAM_M[r])) * (2 / h ** 2) * (1 - np.cos(k * h))
        assert np.allclose(H[sel], c * m[sel], rtol=1e-9, atol=1e-9 * abs(c))
    # uniform magnetisation has no exchange field across the interface either
    assert np.abs(o.ops.exchange(np.tile([0.0, 0.6, 0.8], (o.n, 1)))).max() < 1e-6


# --- implicit midpoint (the paper integrates implicitly, Sec. 2.2) ---------

def test_implicit_midpoint_undamped_macrospin_is_a_cayley_rotation():
    """alpha = 0, uniform m in a fully filled 3D-periodic cell (no exchange or
    demagnetising field), H = H z: x - m = -gamma0 dt ((m + x)/2) x H is the
    Cayley transform of the rotation, i.e. each step turns m about z by
    exactly 2 atan(gamma0 H dt / 2) and keeps its polar angle."""
    p = mg.kuhn_box((3, 3, 3), 2e-9, periodic=0b111, Ms=MS, grid=(12, 12, 12))
    o = model.Oracle(p)
    th0, ph0, Hap, dt, n = 0.9, 0.3, 2e5, 2e-12, 12
    m0 = np.tile([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)], (o.n, 1))
    m, its = o.implicit_midpoint(m0, dt, 0.0, n, h_app=[0.0, 0.0, Hap])
    ph = ph0 + n * 2 * np.arctan(model.GAMMA0 * Hap * dt / 2)
    ex = np.array([np.sin(th0) * np.cos(ph), np.sin(th0) * np.sin(ph), np.cos(th0)])
    assert np.abs(m - ex[None, :]).max() < 1e-9
    # the explicit-rate angle gamma0 H dt per step would be off by far more
    ph_rate = ph0 + n * model.GAMMA0 * Hap * dt
    assert abs(ph_rate - ph) > 1e-4


def test_implicit_midpoint_damped_macrospin_second_order():
    p = mg.kuhn_box((3, 3, 3), 2e-9, periodic=0b111, Ms=MS, grid=(12, 12, 12))
    o = model.Oracle(p)
    A = o.field_matrix()
    th0, ph0, Hap, alpha, T = 0.9, 0.3, 2e5, 0.3, 4e-12
    m0 = np.tile([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)], (o.n, 1))
    g = model.GAMMA0 * Hap / (1 + alpha ** 2)
    th = 2 * np.arctan(np.tan(th0 / 2) * np.exp(-alpha * g * T))
    ph = ph0 + g * T
    ex = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    errs = []
    for n in (4, 8, 16):
        m, _ = o.implicit_midpoint(m0, T / n, alpha, n, h_app=[0.0, 0.0, Hap], A=A)
        errs.append(np.abs(m - ex[None, :]).max())
        assert np.allclose(np.linalg.norm(m, axis=1), 1.0, atol=1e-13)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs


def test_implicit_midpoint_conserves_exchange_energy_without_damping():
    """E_ex = m.K m is quadratic and conserved by the undamped flow, so the
    midpoint rule keeps it to the Newton tolerance (RK4 only to its order),
    and |m| stays 1 with no renormalisation."""
    p = mg.kuhn_box((4, 4, 1), 2e-9, periodic=0b011, jitter=0.2, grid=(12, 12, 4))
    o = model.Oracle(p, with_aim=False)
    m0 = o.unknown_values(p.m)
    e0 = o.ops.exchange_energy(m0)
    m, its = o.implicit_midpoint(m0, 2e-14, 0.0, 10, method="direct", terms=("ex",))
    assert abs(o.ops.exchange_energy(m) - e0) < 1e-11 * abs(e0)
    assert np.allclose(np.linalg.norm(m, axis=1), 1.0, atol=1e-13)
    assert max(its) <= 8
    # RK4 at the same step drifts visibly more
    mr = o.rk4(m0, 2e-14, 0.0, 10, method="direct", terms=("ex",))
    assert abs(o.ops.exchange_energy(mr) - e0) > 100 * abs(o.ops.exchange_energy(m) - e0)


def test_implicit_midpoint_agrees_with_rk4_on_the_film(film):
    """Both rules approximate the same flow: at a step well inside RK4's
    accuracy the two trajectories agree to the midpoint rule's O(dt^2)."""
    o = model.Oracle(film)
    m0 = o.unknown_values(film.m)
    A = o.field_matrix()
    mi, _ = o.implicit_midpoint(m0, 2e-14, 0.5, 10, A=A)
    mi2, _ = o.implicit_midpoint(m0, 1e-14, 0.5, 20, A=A)
    mr = o.rk4(m0, 1e-14, 0.5, 20)
    e1 = np.linalg.norm(mi - mr) / np.linalg.norm(mr - m0)
    e2 = np.linalg.norm(mi2 - mr) / np.linalg.norm(mr - m0)
    assert e2 < e1 / 3.5 and e1 < 1e-2, (e1, e2)
    assert np.allclose(np.linalg.norm(mi, axis=1), 1.0, atol=1e-13)


# --- adaptive midpoint (time-step adaptive predictor-corrector, Sec. 2.2) ---

def _macrospin(alpha, Hap=2e5, th0=0.9, ph0=0.3, T=40e-12):
    """A lone moment in H = Hap z: the rate is gamma0 Hap / (1 + alpha^2),
    the polar angle follows tan(th/2) = tan(th0/2) exp(-alpha g t)."""
    p = mg.kuhn_box((3, 3, 3), 2e-9, periodic=0b111, Ms=MS, Aex=0.0, grid=(12, 12, 12))
    o = model.Oracle(p, with_aim=False)
    A = np.zeros((3 * o.n, 3 * o.n))     # a uniform m in a filled periodic cell: no own field
    m0 = np.tile([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)], (o.n, 1))
    g = model.GAMMA0 * Hap / (1 + alpha ** 2)
    th = 2 * np.arctan(np.tan(th0 / 2) * np.exp(-alpha * g * T))
    ph = ph0 + g * T
    ex = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    return o, A, m0, ex


def test_adaptive_midpoint_estimate_is_the_local_error():
    """Undamped, the right side is linear and a midpoint step turns m by
    exactly 2 atan(x / 2), x = gamma0 H h, where the flow turns it by x: the
    local error of every step is known in closed form, and the estimate
    (predictor constant with non-uniform steps and the history's own errors)
    must reproduce it to leading order."""
    Hap, th0 = 2e5, 0.9
    o, A, m0, ex = _macrospin(0.0, Hap, th0)
    m, info = o.implicit_midpoint_adaptive(m0, 40e-12, 1e-14, 0.0, 1e-8, h_app=[0, 0, Hap], A=A)
    dts = np.array(info["dts"])
    x = model.GAMMA0 * Hap * dts
    true = np.sin(th0) * np.abs(2 * np.arctan(x / 2) - x) / np.sqrt(3)
    est = np.array(info["lte"][2:], dtype=float)
    ratio = est / true[2:]
    assert info["lte"][0] is None and info["lte"][1] is None
    assert np.all(est <= 1e-8)
    assert 0.99 < ratio.min() and ratio.max() < 1.01, (ratio.min(), ratio.max())
    # the steps grew from the first trial step and vary along the run
    assert dts[0] == 1e-14 and dts.max() > 5 * dts[0]
    assert abs(dts.sum() - 40e-12) < 1e-24
    assert np.abs(m - ex[None, :]).max() < 1e-5


def test_adaptive_midpoint_error_follows_the_tolerance():
    """Damped (nonlinear) macrospin against its closed form: each accepted step
    keeps its error near the tolerance and the steps grow as tol^(-1/3), so
    the global error falls as tol^(2/3): a tolerance 8 times smaller gives
    about twice the steps and a quarter of the error."""
    o, A, m0, ex = _macrospin(0.3)
    res = []
    for tol in (1.25e-7, 1.5625e-8):
        m, info = o.implicit_midpoint_adaptive(m0, 40e-12, 1e-14, 0.3, tol, h_app=[0, 0, 2e5],
                                               A=A)
        err = np.abs(m - ex[None, :]).max()
        res.append((len(info["dts"]), err))
        assert err < 2 * len(info["dts"]) * tol
        assert np.allclose(np.linalg.norm(m, axis=1), 1.0, atol=1e-12)
        assert info["rejected"] == 0
    (n1, e1), (n2, e2) = res
    assert 1.7 < n2 / n1 < 2.3, res
    assert 3.2 < e1 / e2 < 4.8, res


def test_adaptive_midpoint_recovers_from_a_failed_newton_step():
    """A first trial step far too long for two Newton iterations is halved
    until Newton converges; the run still meets the closed form."""
    o, A, m0, ex = _macrospin(0.3)
    m, info = o.implicit_midpoint_adaptive(m0, 40e-12, 1e-11, 0.3, 1e-7, h_app=[0, 0, 2e5],
                                           A=A, max_newton=2)
    assert info["rejected"] >= 1 and info["dts"][0] < 1e-11
    assert np.abs(m - ex[None, :]).max() < 1e-4
    with pytest.raises(RuntimeError, match="underflow"):
        o.implicit_midpoint_adaptive(m0, 40e-12, 1e-12, 0.3, 1e-7, h_app=[0, 0, 2e5], A=A,
                                     max_newton=0)


def test_predictor_constant_uniform_steps():
    """Uniform steps: the slope line misses by -h^2 y''' and each slope carries
    (1/24 + 1/12) h^2 y''', which the extrapolation (2 s1 - s2) keeps once,
    so C_p = -1 + 1/8 - 1/24 = -11/12 and Milne's factor C / (C - C_p) = 1/12."""
    cp = model.Oracle.predictor_constant(1.0, 1.0, 1.0)
    assert abs(cp + 11.0 / 12.0) < 1e-15
    c = model.Oracle.LTE_C
    assert abs(c / (c - cp) - 1.0 / 12.0) < 1e-15


# --- adaptive BDF2 (the step-adaptive BDF scheme of the paper's timed run) ---

def test_bdf2_coefficients_are_exact_on_quadratics():
    """The variable-step BDF2 relation x - (a y_n - b y_{n-1}) = beta h y'(t + h)
    holds exactly for y = 1, t and t^2 (its defining property), for uneven
    steps; uniform steps give the textbook 4/3, 1/3, 2/3."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        h, h1 = rng.uniform(0.1, 2.0, size=2)
        a, b, beta = model.Oracle.bdf2_coefficients(h, h1)
        t0, t1, t2 = -h1, 0.0, h
        for k in range(3):
            y = lambda t: t ** k
            dy = k * t2 ** (k - 1) if k else 0.0
            assert abs(y(t2) - (a * y(t1) - b * y(t0)) - beta * h * dy) < 1e-12
    a, b, beta = model.Oracle.bdf2_coefficients(1.0, 1.0)
    assert abs(a - 4 / 3) < 1e-15 and abs(b - 1 / 3) < 1e-15 and abs(beta - 2 / 3) < 1e-15
    assert model.Oracle.bdf2_estimate_factor(1.0, 1.0, 1.0) == pytest.approx(1 / 3)


def test_bdf2_estimate_is_the_local_error():
    """Undamped macrospin (linear right side): the true local error of each
    accepted step is the distance of the new state from the current one
    turned by gamma0 H h about z. Past the start (a backward-Euler step,
    whose error is not smooth in the history, makes the first estimates
    conservative) and before the shortened last step, the estimate equals it
    to leading order."""
    Hap, th0 = 2e5, 0.9
    o, A, m0, ex = _macrospin(0.0, Hap, th0)
    m, info = o.implicit_bdf2_adaptive(m0, 40e-12, 1e-14, 0.0, 1e-8, h_app=[0, 0, Hap], A=A,
                                       record=True)
    st = info["states"]
    ratios = []
    for k, h in enumerate(info["dts"]):
        if info["lte"][k] is None:
            continue
        ang = model.GAMMA0 * Hap * h
        R = np.array([[np.cos(ang), -np.sin(ang), 0], [np.sin(ang), np.cos(ang), 0], [0, 0, 1]])
        true = np.linalg.norm(st[k + 1][0] - R @ st[k][0]) / np.sqrt(3)
        ratios.append(info["lte"][k] / true)
    ratios = np.array(ratios)
    assert np.all(ratios[:8] >= 0.95)
    mid = ratios[8:-1]
    assert mid.size > 300 and 0.97 < mid.min() and mid.max() < 1.03, (mid.min(), mid.max())
    assert np.abs(m - ex[None, :]).max() < 1e-5


def test_bdf2_error_follows_the_tolerance():
    """Damped macrospin against its closed form: a tolerance 8 times smaller
    gives about twice the steps and a quarter of the error."""
    o, A, m0, ex = _macrospin(0.3)
    res = []
    for tol in (1.25e-7, 1.5625e-8):
        m, info = o.implicit_bdf2_adaptive(m0, 40e-12, 1e-14, 0.3, tol, h_app=[0, 0, 2e5], A=A)
        res.append((len(info["dts"]), np.abs(m - ex[None, :]).max()))
        assert np.allclose(np.linalg.norm(m, axis=1), 1.0, atol=1e-12)
    (n1, e1), (n2, e2) = res
    assert 1.7 < n2 / n1 < 2.3, res
    assert 3.2 < e1 / e2 < 4.8, res
