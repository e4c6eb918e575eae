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
