"""Pins of the oracle's AIM (paper Sec. 3.2.2, steps 1-4).

* Charges and observers on grid points: projection and interpolation are
  identities, so steps 1-3 must equal the direct sum with the sampled PGF
  (pins the grid kernel, the FFT convolution and the zero padding).
* The Lagrange weights reproduce polynomials of degree <= p.
* With the "full" correction (the whole PGF subtracted and added back for
  every pair) the AIM equals the direct point-charge sum to rounding.
* The AIM operator is symmetric.
* The AIM error against the direct sum falls when the stencil order or the
  near-region radius grows.
"""
import numpy as np
import pytest

from oracle import aim, pgf as P, model
from paper_2409_13958_amd import meshgen as mg

GRIDS = [
    ("3d", 0b111, np.array([1.0, 1.2, 0.9]), (12, 14, 11)),
    ("2d", 0b011, np.array([1.0, 1.2, 0.0]), (12, 12, 6)),
    ("1d", 0b100, np.array([0.0, 0.0, 1.3]), (7, 6, 16)),
]


def _grid_points(mask, L, N, n, rng):
    """n random grid points; on non-periodic axes the extreme points are included
    so that the bounding box spans the grid."""
    N = np.array(N)
    idx = np.stack([rng.integers(0, N[a], n) for a in range(3)], axis=1)
    for a in range(3):
        if not (mask >> a) & 1:
            idx[0, a], idx[1, a] = 0, N[a] - 1
    delta = np.where([(mask >> a) & 1 for a in range(3)], L / N, 0.37 + 0.05 * np.arange(3))
    idx = np.unique(idx, axis=0)
    return idx * delta, idx, delta


@pytest.mark.parametrize("name,mask,L,N", GRIDS)
def test_grid_points_equal_direct_grid_sum(name, mask, L, N):
    rng = np.random.default_rng(11)
    pos, idx, delta = _grid_points(mask, L, N, 40, rng)
    A = aim.AIM(pos, mask, L, N, order_p=3, near_boxes=1)
    assert np.allclose(A.grid.delta, delta)
    q = rng.standard_normal(pos.shape[0])
    q -= q.mean()
    ut = A.interpolate(A.convolve(A.project(q)))
    d = pos[:, None, :] - pos[None, :, :]
    G = np.empty((pos.shape[0], pos.shape[0]))
    off = ~np.eye(pos.shape[0], dtype=bool)
    G[off] = P.pgf(d[off], mask, L)
    G[~off] = P.greg0(mask, L)
    assert np.allclose(ut, G @ q, rtol=0, atol=1e-12 * np.abs(G @ q).max())


@pytest.mark.parametrize("name,mask,L,N", GRIDS)
def test_lagrange_reproduces_cubics(name, mask, L, N):
    rng = np.random.default_rng(12)
    N = np.array(N)
    g = aim.Grid(np.array([[0, 0, 0], [1, 1, 1]]) * np.where(
        [(mask >> a) & 1 for a in range(3)], 0.0, (N - 1) * 0.3), mask, L, N, order_p=3)
    # points away from periodic wrap so that a plain cubic in the index is valid
    s = rng.uniform(2.0, np.minimum(N - 3.0, 8.0), (50, 3))
    pos = g.origin + s * g.delta
    s2, b, st, w = g.locate(pos)
    W = g.stencil_weights(w)
    offs = np.arange(4)
    I = np.stack(np.meshgrid(offs, offs, offs, indexing="ij"), axis=-1).reshape(-1, 3)
    gidx = st[:, None, :] + I[None, :, :]

    def f(x):
        return 1.3 * x[..., 0] ** 3 - 0.7 * x[..., 1] ** 2 * x[..., 2] + 2 * x[..., 2] ** 3 + 0.1
    assert np.allclose(np.sum(W * f(gidx.astype(float)), axis=1), f(s2), rtol=1e-12)
    assert np.allclose(W.sum(axis=1), 1.0, atol=1e-13)


@pytest.mark.parametrize("name,mask,L,N", GRIDS)
def test_full_correction_equals_direct_sum(name, mask, L, N):
    rng = np.random.default_rng(13)
    n = 30
    span = np.where([(mask >> a) & 1 for a in range(3)], L, 2.0)
    pos = rng.uniform(0, 1, (n, 3)) * span
    A = aim.AIM(pos, mask, L, N, order_p=3, near_boxes=1)
    q = rng.standard_normal(n)
    q -= q.mean()
    u = A.potential(q, full=True) * 4 * np.pi
    d = pos[:, None, :] - pos[None, :, :]
    G = np.empty((n, n))
    off = ~np.eye(n, dtype=bool)
    G[off] = P.pgf(d[off], mask, L)
    G[~off] = P.greg0(mask, L)
    assert np.allclose(u, G @ q, rtol=0, atol=1e-11 * np.abs(G @ q).max())


def test_aim_operator_symmetric():
    p = mg.kuhn_box((5, 5, 2), 1.0, periodic=0b011, jitter=0.2, grid=(12, 12, 5))
    o = model.Oracle(p)
    A = o.aim
    rng = np.random.default_rng(14)
    q1, q2 = rng.standard_normal((2, o.n))
    P_all = A.precorrection(np.arange(o.n))

    def S(q):
        return A.interpolate(A.convolve(A.project(q))) + P_all @ q
    assert q2 @ S(q1) == pytest.approx(q1 @ S(q2), rel=1e-12)


def test_precorrection_removes_grid_g0_for_self_pair():
    """P_nn = -W_n^T K0 W_n (no exact G0 for the self pair)."""
    p = mg.kuhn_box((4, 4, 4), 1.0, periodic=0b111, jitter=0.2, grid=(12, 12, 12))
    o = model.Oracle(p)
    A = o.aim
    Pm = A.precorrection(np.array([3]))
    g = A.grid
    offs = np.arange(4)
    I = np.stack(np.meshgrid(offs, offs, offs, indexing="ij"), axis=-1).reshape(-1, 3)
    w = A.W3[3]
    k0 = 0.0
    for i in range(64):
        for j in range(64):
            d = (I[i] - I[j]) * g.delta
            r = np.linalg.norm(d)
            if r > 0:
                k0 += w[i] * w[j] / r
    assert Pm[0, 3] == pytest.approx(-k0, rel=1e-12)


def test_aim_error_falls_with_order_and_radius():
    """Far pairs are interpolated across both stencils, so the near region has
    to grow with the stencil: at fixed p the error falls with r_b, and once
    r_b exceeds p it falls with p as well."""
    p = mg.kuhn_box((6, 6, 2), 1.0, periodic=0b011, jitter=0.2, grid=(24, 24, 6))
    rng = np.random.default_rng(15)
    errs = {}
    ref = None
    for (pp, rb) in [(3, 2), (3, 3), (3, 4), (3, 5), (1, 5), (5, 5)]:
        o = model.Oracle(p, order_p=pp, near_boxes=rb)
        if ref is None:
            m = rng.standard_normal((o.n, 3))
            ref = o.potential(m, method="direct", z0=False)
        u = o.potential(m, method="aim", z0=False)
        errs[(pp, rb)] = np.linalg.norm(u - ref) / np.linalg.norm(ref)
    assert errs[(3, 2)] > errs[(3, 3)] > errs[(3, 4)] > errs[(3, 5)]
    assert errs[(1, 5)] > errs[(3, 5)] > errs[(5, 5)]
    assert errs[(3, 2)] < 5e-2 and errs[(5, 5)] < 1e-3
