"""Pins of the oracle's periodic bookkeeping and P1 operators (paper Secs. 2.2, 3.1, 3.2.1).

Closed forms used (derived, not from the paper): on an unjittered Kuhn
(6-tetrahedra) lattice the P1 stiffness couples only axis neighbours, so
-K/mu is the 7-point finite-difference Laplacian, also on film faces where
mass and in-plane stiffness are both halved.
"""
import json
import os

import numpy as np
import pytest

from oracle import periodic, fem, model
from paper_2409_13958_amd import meshgen as mg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def brute_pairs(xyz, mask, L, tol):
    """O(N^2) search over all lattice offsets in {-2..2}^d."""
    per = [a for a in range(3) if (mask >> a) & 1]
    offs = np.stack(np.meshgrid(*[np.arange(-2, 3) if a in per else np.array([0])
                                  for a in range(3)], indexing="ij"), -1).reshape(-1, 3)
    out = set()
    for i in range(xyz.shape[0]):
        for o in offs:
            d = np.linalg.norm(xyz - (xyz[i] + o * L), axis=1)
            for j in np.nonzero(d < tol)[0]:
                if j != i:
                    out.add((min(i, int(j)), max(i, int(j))))
    return out


def test_pairs_match_brute_force_and_c1_count():
    p = mg.film_c1()
    pairs = periodic.pbc_pairs(p.xyz, p.periodic, p.L)
    got = set((min(a, b), max(a, b)) for a, b in pairs.tolist())
    assert got == brute_pairs(p.xyz, p.periodic, p.L, 1e-15)
    uk, reps, npairs = periodic.unknowns(p.xyz, p.periodic, p.L)
    assert reps.size == 200 and p.xyz.shape[0] - reps.size == 42
    # representatives are the smallest index of their class
    for n in range(p.xyz.shape[0]):
        assert reps[uk[n]] <= n


def test_pairs_across_combined_shifts():
    """Images that differ by several periods at once, with no single-axis
    image in the mesh, still merge (protruding cells produce them)."""
    L = np.array([1.0, 1.0, 1.0])
    xyz = np.array([[0.2, 0.3, 0.4], [1.2, -0.7, 0.4], [0.2, 0.3, 2.4], [0.5, 0.5, 0.5]])
    uk, reps, _ = periodic.unknowns(xyz, 0b111, L)
    assert uk[0] == uk[1] == uk[2] and uk[3] != uk[0]
    uk2, _, _ = periodic.unknowns(xyz, 0b011, L)
    assert uk2[0] == uk2[1] and uk2[2] != uk2[0]


def test_corner_class_has_eight_members():
    """Sec. 2.2: a corner of a 3D-periodic cube has up to 7 children."""
    p = mg.kuhn_box((3, 3, 3), 1.0, periodic=0b111)
    uk, reps, _ = periodic.unknowns(p.xyz, p.periodic, p.L)
    counts = np.bincount(uk)
    assert counts.max() == 8 and np.sum(counts == 8) == 1
    assert reps.size == 27


def test_remap_protruding_parallelogram():
    """Sec. 4.1 example: a 1D x-periodic parallelogram with L_x = 2, D_x = 3
    is folded into a rectangle of width L_x by Eq. shift_hms."""
    with open(os.path.join(GOLDEN, "protruding_parallelogram.json")) as f:
        g = json.load(f)
    pts = np.array(g["points"], dtype=np.float64)
    L = np.array([g["Lx"], 0.0, 0.0])
    assert np.ptp(pts[:, 0]) == pytest.approx(g["Dx"])
    out = periodic.remap(pts, 0b001, L)
    r0 = pts.mean(axis=0)
    assert np.all(out[:, 0] >= r0[0] - L[0] / 2 - 1e-12)
    assert np.all(out[:, 0] < r0[0] + L[0] / 2 + 1e-12)
    assert np.ptp(out[:, 0]) <= L[0] + 1e-12
    shift = (out[:, 0] - pts[:, 0]) / L[0]
    assert np.allclose(shift, np.round(shift))
    assert np.array_equal(out[:, 1:], pts[:, 1:])


def _ops(p):
    uk, reps, _ = periodic.unknowns(p.xyz, p.periodic, p.L)
    return fem.LocalOperators(p.xyz, p.tets.astype(np.int64), p.region, p.Ms, p.Aex, uk,
                              reps.size), uk, reps


def test_exchange_uniform_zero_and_symmetric():
    p = mg.kuhn_box((4, 4, 3), 1e-9, periodic=0b011, jitter=0.2)
    ops, uk, reps = _ops(p)
    m = np.tile([0.6, 0.0, 0.8], (reps.size, 1))
    scale = np.abs(ops.exchange(np.random.default_rng(4).standard_normal((reps.size, 3)))).max()
    assert np.abs(ops.exchange(m)).max() < 1e-12 * scale
    assert abs(ops.K - ops.K.T).max() < 1e-12 * abs(ops.K).max()


def test_exchange_cosine_wave_closed_form():
    h = 2e-9
    p = mg.kuhn_box((10, 10, 1), h, periodic=0b011, Ms=8e5, Aex=1.3e-11)
    ops, uk, reps = _ops(p)
    x = p.xyz[reps, 0]
    k = 2 * np.pi * 2 / p.L[0]
    m = np.stack([np.cos(k * x), np.sin(k * x), np.zeros_like(x)], axis=1)
    H = ops.exchange(m)
    coef = -(2 * 1.3e-11 / (fem.MU0 * 8e5)) * (2 / h ** 2) * (1 - np.cos(k * h))
    assert np.allclose(H, coef * m, rtol=1e-12, atol=1e-12 * abs(coef))


def test_exchange_energy_derivative():
    """H_ex = -(1/(mu0 mu_n)) dE_ex/dm_n (central differences)."""
    p = mg.kuhn_box((3, 3, 2), 1e-9, periodic=0b001, jitter=0.2)
    ops, uk, reps = _ops(p)
    rng = np.random.default_rng(5)
    m = rng.standard_normal((reps.size, 3))
    H = ops.exchange(m)
    eps = 1e-3
    for n, c in [(0, 0), (5, 2), (reps.size - 1, 1)]:
        mp, mm = m.copy(), m.copy()
        mp[n, c] += eps
        mm[n, c] -= eps
        dE = (ops.exchange_energy(mp) - ops.exchange_energy(mm)) / (2 * eps)
        assert H[n, c] == pytest.approx(-dE / (fem.MU0 * ops.mu[n]), rel=1e-8)


def test_charges_sum_zero_and_uniform_cases():
    rng = np.random.default_rng(6)
    p = mg.kuhn_box((4, 4, 4), 1e-9, periodic=0b111, jitter=0.2)
    ops, uk, reps = _ops(p)
    m = rng.standard_normal((reps.size, 3))
    q = ops.charges(m)
    assert abs(q.sum()) < 1e-12 * np.abs(q).sum()
    # uniform m in a fully filled 3D-periodic cell carries no charge
    assert np.abs(ops.charges(np.tile([0.3, -0.5, 0.8], (reps.size, 1)))).max() \
        < 1e-12 * np.abs(q).max()
    # in-plane uniform m in a 2D-periodic film carries no charge
    f = mg.kuhn_box((4, 4, 2), 1e-9, periodic=0b011, jitter=0.0)
    ops2, _, r2 = _ops(f)
    assert np.abs(ops2.charges(np.tile([0.6, 0.8, 0.0], (r2.size, 1)))).max() < 1e-12 * 8e5 * 1e-18
    # out of plane: only the two faces, equal and opposite
    qz = ops2.charges(np.tile([0.0, 0.0, 1.0], (r2.size, 1)))
    zf = f.xyz[r2, 2]
    top, bot = qz[zf > zf.max() - 1e-12].sum(), qz[zf < zf.min() + 1e-12].sum()
    assert top == pytest.approx(8e5 * f.L[0] * f.L[1], rel=1e-12)
    assert bot == pytest.approx(-8e5 * f.L[0] * f.L[1], rel=1e-12)


def test_gradient_exact_for_linear_potential():
    """H = -(1/mu) D^T u reproduces -grad u for u linear in the non-periodic axis."""
    f = mg.kuhn_box((4, 4, 3), 1e-9, periodic=0b011, jitter=0.2)
    ops, uk, reps = _ops(f)
    c = 3.7e5
    u = c * f.xyz[reps, 2]
    H = ops.gradient_field(u)
    assert np.allclose(H, np.tile([0, 0, -c], (reps.size, 1)), rtol=0, atol=1e-9 * c)


def test_gradient_mu_weighted_sum_vanishes_in_filled_cell():
    p = mg.kuhn_box((4, 4, 4), 1e-9, periodic=0b111, jitter=0.2)
    ops, uk, reps = _ops(p)
    u = np.random.default_rng(7).standard_normal(reps.size)
    H = ops.gradient_field(u)
    assert np.abs((ops.mu[:, None] * H).sum(axis=0)).max() < 1e-12 * np.abs(ops.mu[:, None] * H).sum()


def test_charges_transpose_of_gradient():
    """q'.u = -sum_n mu_n m_n . H[u]: the charge and gradient operators are adjoint."""
    p = mg.kuhn_box((3, 3, 3), 1e-9, periodic=0b101, jitter=0.2)
    ops, uk, reps = _ops(p)
    rng = np.random.default_rng(8)
    m = rng.standard_normal((reps.size, 3))
    u = rng.standard_normal(reps.size)
    lhs = ops.charges(m) @ u
    rhs = -np.sum(ops.mu[:, None] * m * ops.gradient_field(u))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_mean_edge_length_structured():
    p = mg.kuhn_box((2, 2, 2), 1.0)
    # unit cube edges: axis (1), face diagonals (sqrt 2), body diagonal (sqrt 3)
    hb = model.mean_edge_length(p.xyz, p.tets)
    assert 1.0 < hb < np.sqrt(3)
