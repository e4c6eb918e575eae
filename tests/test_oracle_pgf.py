"""Pins of the oracle's periodic Green's function (paper Eq. 2, k0 = 0).

The Ewald forms are checked against things they do not contain: the
brute-force lattice sum of 1/r (differences converge), the Laplacian of
the lattice of unit charges, reflection symmetry, periodicity, the far-field
asymptotes and independence from the splitting parameter.
"""
import numpy as np
import pytest

from oracle import pgf as P

CASES = [
    ("3d", 0b111, np.array([1.0, 1.3, 0.8])),
    ("2d", 0b011, np.array([1.0, 1.3, 0.0])),
    ("2d_xz", 0b101, np.array([1.1, 0.0, 0.9])),
    ("1d_z", 0b100, np.array([0.0, 0.0, 1.2])),
    ("1d_x", 0b001, np.array([2.0, 0.0, 0.0])),
]


@pytest.mark.parametrize("name,mask,L", CASES)
def test_eta_independence(name, mask, L):
    rng = np.random.default_rng(1)
    r = rng.uniform(-1.5, 1.5, (12, 3))
    e0 = P.default_eta(mask, L)
    g = [P.pgf(r, mask, L, e0 * f) for f in (0.6, 1.0, 1.8)]
    scale = np.abs(g[1]).max()
    assert np.max(np.abs(g[0] - g[1])) < 1e-13 * scale
    assert np.max(np.abs(g[2] - g[1])) < 1e-13 * scale
    r0 = [P.greg0(mask, L, e0 * f) for f in (0.6, 1.0, 1.8)]
    assert abs(r0[0] - r0[1]) < 1e-13 * abs(r0[1]) and abs(r0[2] - r0[1]) < 1e-13 * abs(r0[1])


@pytest.mark.parametrize("name,mask,L", CASES)
def test_periodicity_and_reflection(name, mask, L):
    rng = np.random.default_rng(2)
    r = rng.uniform(-0.6, 0.6, (8, 3))
    g = P.pgf(r, mask, L)
    for a in range(3):
        if (mask >> a) & 1:
            s = r.copy()
            s[:, a] += 2 * L[a]
            assert np.allclose(P.pgf(s, mask, L), g, rtol=1e-13, atol=0)
        f = r.copy()
        f[:, a] = -f[:, a]
        assert np.allclose(P.pgf(f, mask, L), g, rtol=1e-13, atol=0)


@pytest.mark.parametrize("name,mask,L", CASES)
def test_regular_part_at_origin(name, mask, L):
    """G_reg(0) = lim_{r->0} (G^p(r) - 1/r)."""
    d = np.array([[0.7, -0.4, 0.5]]) * 1e-4 * L.max()
    g = P.pgf(d, mask, L)[0] - 1.0 / np.linalg.norm(d)
    assert abs(g - P.greg0(mask, L)) < 1e-7 * abs(P.greg0(mask, L))


@pytest.mark.parametrize("name,mask,L", CASES)
def test_laplacian_away_from_lattice(name, mask, L):
    """FD Laplacian: 4 pi / V in 3D (uniform neutralising background), 0 in 1D/2D."""
    rng = np.random.default_rng(3)
    r = rng.uniform(0.2, 0.4, (4, 3)) * L.max()

    def lap(h):
        out = -6 * P.pgf(r, mask, L)
        for a in range(3):
            for s in (-1, 1):
                rr = r.copy()
                rr[:, a] += s * h
                out += P.pgf(rr, mask, L)
        return out / (h * h)
    h = 1e-2 * L.max()
    rich = (4 * lap(h / 2) - lap(h)) / 3          # removes the O(h^2) error
    expect = 4 * np.pi / np.prod(L) if mask == 0b111 else 0.0
    # a scale that is finite for every periodicity: 4 pi / L_max^3 is the
    # 3D background density for a cube of the largest period (12.1 for the
    # 3D case here, 1.6 - 9.4 for the others); the residuals are ~3e-7, and
    # dropping the 2D/1D far-field or background terms moves them to O(1)
    scale = 4 * np.pi / L.max() ** 3
    assert np.all(np.isfinite(rich))
    assert np.allclose(rich, expect, rtol=0, atol=1e-6 * scale)


def test_lattice_sum_1d():
    mask, L = 0b100, np.array([0.0, 0.0, 1.2])
    r = np.array([[0.3, -0.2, 0.25], [-0.1, 0.35, -0.4]])
    g = P.pgf(r, mask, L)
    s = P.lattice_sum(r, mask, L, 2000.0)
    assert abs((s[0] - s[1]) - (g[0] - g[1])) < 1e-6


def test_lattice_sum_2d_disc():
    """Disc partial sums converge like 1/R; Richardson removes that term."""
    mask, L = 0b011, np.array([1.0, 1.3, 0.0])
    r = np.array([[0.3, -0.2, 0.25], [-0.1, 0.35, -0.4]])
    g = P.pgf(r, mask, L)
    s1 = P.lattice_sum(r, mask, L, 60.0)
    s2 = P.lattice_sum(r, mask, L, 120.0)
    rich = 2 * (s2[0] - s2[1]) - (s1[0] - s1[1])
    assert abs(rich - (g[0] - g[1])) < 2e-4 * abs(g[0] - g[1])


def test_lattice_sum_3d_sphere():
    """Spherical partial sums carry the depolarisation term -(2 pi/3V)|r|^2
    relative to the zero-mean (tin-foil) Ewald sum."""
    mask, L = 0b111, np.array([1.0, 1.3, 0.8])
    r = np.array([[0.3, -0.2, 0.25], [-0.1, 0.35, -0.3]])
    g = P.pgf(r, mask, L)
    V = np.prod(L)
    ex = (g[0] - g[1]) - 2 * np.pi / (3 * V) * (r[0] @ r[0] - r[1] @ r[1])
    s = np.mean([np.diff(P.lattice_sum(r, mask, L, R))[0] * -1 for R in (24.0, 25.0, 26.0, 27.0)])
    assert abs(s - ex) < 2e-3 * abs(ex)
    # without the depolarisation term the sums would disagree clearly
    assert abs(s - (g[0] - g[1])) > 20 * abs(s - ex)


def test_far_field_2d():
    mask, L = 0b011, np.array([1.0, 1.3, 0.0])
    A = L[0] * L[1]
    z = np.array([5.0, 6.0])
    r = np.stack([[0.2, 0.1, z[0]], [0.2, 0.1, z[1]]])
    g = P.pgf(r, mask, L)
    # -2 pi |z| / A plus exponentially small terms
    assert abs((g[1] - g[0]) - (-2 * np.pi / A) * (z[1] - z[0])) < 1e-8


def test_far_field_1d():
    mask, L = 0b001, np.array([2.0, 0.0, 0.0])
    rho = np.array([12.0, 20.0])
    r = np.stack([[0.3, rho[0], 0.0], [0.3, 0.0, rho[1]]])
    g = P.pgf(r, mask, L)
    assert abs((g[1] - g[0]) - (-2.0 / L[0]) * np.log(rho[1] / rho[0])) < 1e-8


def test_free_space_limit_small_distance():
    """Near the origin the PGF is 1/r plus a smooth remainder."""
    for mask, L in [(0b111, np.array([1.0, 1.0, 1.0])), (0b011, np.array([1.0, 1.0, 0.0]))]:
        r = np.array([[1e-3, 0, 0], [2e-3, 0, 0]])
        g = P.pgf(r, mask, L)
        assert abs((g[0] - g[1]) - (1e3 - 5e2)) < 1e-5
