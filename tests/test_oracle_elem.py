"""Pins of the oracle's element-exact integrals (correction matrix of Eq. hms_d2b).

A cube split into its six Kuhn tetrahedra is compared with closed forms:
int 1/R over a box, int 1/R and int x/R over a rectangle, at observers on
cube corners (singular, Duffy path) and off the cube (adaptive path). The
dipole-form integral of a linearly magnetised tetrahedron is a third,
independent route that must agree with volume plus surface charges.
"""
import numpy as np
import pytest

from oracle import elem, fem
from paper_2409_13958_amd import meshgen as mg


def _F0(X, Y, Z):
    """Corner function of int int dX dY / R."""
    R = np.sqrt(X * X + Y * Y + Z * Z)
    with np.errstate(all="ignore"):
        t1 = np.where(X == 0, 0.0, X * np.log(Y + R))
        t2 = np.where(Y == 0, 0.0, Y * np.log(X + R))
        t3 = np.where(Z == 0, 0.0, Z * np.arctan(X * Y / (Z * R)))
    return t1 + t2 - t3


def _F1(X, Y, Z):
    """Corner function of int int X dX dY / R."""
    R = np.sqrt(X * X + Y * Y + Z * Z)
    with np.errstate(all="ignore"):
        lg = np.where(X * X + Z * Z == 0, 0.0, (X * X + Z * Z) * np.log(Y + R))
    return 0.5 * (Y * R + lg)


def _rect(F, x1, x2, y1, y2, z0, r):
    X1, X2, Y1, Y2, Z = x1 - r[0], x2 - r[0], y1 - r[1], y2 - r[1], z0 - r[2]
    return F(X2, Y2, Z) - F(X1, Y2, Z) - F(X2, Y1, Z) + F(X1, Y1, Z)


def _cube():
    p = mg.kuhn_box((1, 1, 1), 1.0)
    V, g = fem.tet_geometry(p.xyz, p.tets)
    return p.xyz, p.tets, g


def _coeffs(r, xyz, tets, g):
    X = xyz[tets]
    vert = np.full(tets.shape[0], -1)
    for e in range(tets.shape[0]):
        hit = np.nonzero(np.linalg.norm(X[e] - r, axis=1) < 1e-12)[0]
        if hit.size:
            vert[e] = hit[0]
    return elem.element_coeffs(np.repeat(r[None], tets.shape[0], 0), X, g, vert)


OBS = [(0, 0, 0), (1, 1, 1), (1, 0, 0), (0, 1, 1), (1, 1, 0), (1.3, 0.2, 0.4),
       (0.5, 0.5, 1.05), (0.2, 0.3, -0.05), (-0.7, 1.4, 2.1), (3.0, -2.0, 0.5)]


@pytest.mark.parametrize("r", OBS)
def test_uniform_cube_z(r):
    """M = z-hat: charges +1 on the top face, -1 on the bottom face."""
    r = np.array(r, dtype=np.float64)
    xyz, tets, g = _cube()
    C = _coeffs(r, xyz, tets, g)
    u = C[:, :, 2].sum()                   # 4 pi u / Ms with m_j = z-hat
    ex = _rect(_F0, 0, 1, 0, 1, 1, r) - _rect(_F0, 0, 1, 0, 1, 0, r)
    assert u == pytest.approx(ex, abs=1e-9)


@pytest.mark.parametrize("r", OBS)
def test_linear_cube(r):
    """M = x z-hat (div M = 0): charges +x on the top face, -x on the bottom."""
    r = np.array(r, dtype=np.float64)
    xyz, tets, g = _cube()
    C = _coeffs(r, xyz, tets, g)
    xj = xyz[tets][:, :, 0]                 # m_j = (0, 0, x_j)
    u = np.sum(C[:, :, 2] * xj)
    top = _rect(_F1, 0, 1, 0, 1, 1, r) + r[0] * _rect(_F0, 0, 1, 0, 1, 1, r)
    bot = _rect(_F1, 0, 1, 0, 1, 0, r) + r[0] * _rect(_F0, 0, 1, 0, 1, 0, r)
    assert u == pytest.approx(top - bot, abs=1e-9)


@pytest.mark.parametrize("r", OBS)
def test_volume_charge_cube(r):
    """M = (x, 0, 0): volume charge -1, surface charge x on the x = 1 face."""
    r = np.array(r, dtype=np.float64)
    xyz, tets, g = _cube()
    C = _coeffs(r, xyz, tets, g)
    xj = xyz[tets][:, :, 0]
    u = np.sum(C[:, :, 0] * xj)
    # u = oint sigma / R - int 1/R dV with sigma = 1 on x = 1 only
    face = _rect_x(1.0, r)
    vol = _volume_reference(r)
    assert u == pytest.approx(face - vol, abs=1e-8)


def _rect_x(x0, r):
    # face x = x0, coordinates (y, z): int int 1/R over the unit square
    rr = np.array([r[1], r[2], r[0]])
    return _rect(_F0, 0, 1, 0, 1, x0, rr)


def _volume_reference(r):
    """int over the unit cube of 1/|r - r'| from the closed-form box integral;
    an observer on the cube splits it into boxes cornered at r."""
    if np.all((r >= -1e-12) & (r <= 1 + 1e-12)):
        # observer on the cube: split the cube at r into boxes with r at a corner,
        # where int_box 1/R has the closed-form corner function below
        tot = 0.0
        for xa, xb in ((0.0, r[0]), (r[0], 1.0)):
            for ya, yb in ((0.0, r[1]), (r[1], 1.0)):
                for za, zb in ((0.0, r[2]), (r[2], 1.0)):
                    tot += _box_int(xa, xb, ya, yb, za, zb, r)
        return tot
    return _box_int(0, 1, 0, 1, 0, 1, r)


def _box_int(x1, x2, y1, y2, z1, z2, r):
    """Closed form of int_box 1/R (corner function of the uniform box potential)."""
    def G(X, Y, Z):
        R = np.sqrt(X * X + Y * Y + Z * Z)
        with np.errstate(all="ignore"):
            a = np.where((Y == 0) | (Z == 0), 0.0, Y * Z * np.log(X + R))
            b = np.where((X == 0) | (Z == 0), 0.0, X * Z * np.log(Y + R))
            c = np.where((X == 0) | (Y == 0), 0.0, X * Y * np.log(Z + R))
            d = np.where(X == 0, 0.0, 0.5 * X * X * np.arctan(Y * Z / (X * R)))
            e = np.where(Y == 0, 0.0, 0.5 * Y * Y * np.arctan(X * Z / (Y * R)))
            f = np.where(Z == 0, 0.0, 0.5 * Z * Z * np.arctan(X * Y / (Z * R)))
        return a + b + c - d - e - f
    if x2 - x1 <= 0 or y2 - y1 <= 0 or z2 - z1 <= 0:
        return 0.0
    tot = 0.0
    for sx, X in ((1, x2 - r[0]), (-1, x1 - r[0])):
        for sy, Y in ((1, y2 - r[1]), (-1, y1 - r[1])):
            for sz, Z in ((1, z2 - r[2]), (-1, z1 - r[2])):
                tot += sx * sy * sz * G(X, Y, Z)
    return float(tot)


def test_box_integral_closed_form_against_quadrature():
    """The volume closed form used above, checked by plain Gauss-Legendre."""
    r = np.array([2.5, -1.0, 0.3])
    x, w = np.polynomial.legendre.leggauss(40)
    x, w = 0.5 * (x + 1), 0.5 * w
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    W = w[:, None, None] * w[None, :, None] * w[None, None, :]
    q = np.sum(W / np.sqrt((X - r[0]) ** 2 + (Y - r[1]) ** 2 + (Z - r[2]) ** 2))
    assert _box_int(0, 1, 0, 1, 0, 1, r) == pytest.approx(q, rel=1e-12)


def test_far_element_is_a_dipole():
    xyz, tets, g = _cube()
    pts = xyz[tets[2]] * 0.3
    X = pts[None]
    V, gg = fem.tet_geometry(pts, np.arange(4)[None])
    r = np.array([[40.0, -25.0, 31.0]])
    C = elem.element_coeffs(r, X, gg, np.array([-1]))
    c = X[0].mean(axis=0)
    d = r[0] - c
    dip = V[0] * d / np.linalg.norm(d) ** 3       # sum_j C_j for uniform m
    assert np.allclose(C[0].sum(axis=0), dip, rtol=1e-6)


def _cube_boundary_triangles(xyz, tets, axis, value):
    """Triangles (vertex coordinates) of the cube face {x_axis = value}."""
    out = []
    for t in tets:
        for a in range(4):
            tri = np.delete(t, a)
            if np.all(np.abs(xyz[tri, axis] - value) < 1e-12):
                out.append(xyz[tri])
    return np.array(out)


@pytest.mark.parametrize("r", OBS)
def test_tet_inv_r_sums_to_box(r):
    r = np.array(r, dtype=np.float64)
    xyz, tets, g = _cube()
    X = xyz[tets]
    vert = np.array([next((i for i in range(4) if np.linalg.norm(X[e, i] - r) < 1e-12), -1)
                     for e in range(6)])
    I = elem.tet_inv_r(np.repeat(r[None], 6, 0), X, vert)
    assert I.sum() == pytest.approx(_volume_reference(r), abs=1e-9)


@pytest.mark.parametrize("r", OBS)
def test_triangle_integrals_on_top_face(r):
    r = np.array(r, dtype=np.float64)
    xyz, tets, g = _cube()
    T = _cube_boundary_triangles(xyz, tets, 2, 1.0)
    assert T.shape[0] == 2
    vert = np.array([next((i for i in range(3) if np.linalg.norm(T[e, i] - r) < 1e-12), -1)
                     for e in range(T.shape[0])])
    I = elem.tri_lambda_inv_r(np.repeat(r[None], T.shape[0], 0), T, vert)   # [2,3]
    # constant density: sum of the three weights
    assert I.sum() == pytest.approx(_rect(_F0, 0, 1, 0, 1, 1, r), abs=1e-9)
    # density x: nodal values times weights
    lin = np.sum(I * T[:, :, 0])
    ex = _rect(_F1, 0, 1, 0, 1, 1, r) + r[0] * _rect(_F0, 0, 1, 0, 1, 1, r)
    assert lin == pytest.approx(ex, abs=1e-9)


@pytest.mark.parametrize("r", [(0, 0, 0), (1, 0, 1), (1.4, 0.3, 0.6), (0.5, -0.3, 0.2)])
def test_dipole_form_equals_volume_plus_surface(r):
    """Linear M over the cube: dipole-form integrals vs volume + surface charges."""
    r = np.array(r, dtype=np.float64)
    xyz, tets, g = _cube()
    X = xyz[tets]
    rng = np.random.default_rng(31)
    A = rng.standard_normal((3, 3))
    b = rng.standard_normal(3)
    mj = xyz @ A.T + b                       # m(x) = A x + b, linear: exact in P1
    C = _coeffs(r, xyz, tets, g)
    dip = np.einsum("eji,eji->", C, mj[tets])
    vert = np.array([next((i for i in range(4) if np.linalg.norm(X[e, i] - r) < 1e-12), -1)
                     for e in range(6)])
    vol = -np.trace(A) * elem.tet_inv_r(np.repeat(r[None], 6, 0), X, vert).sum()
    surf = 0.0
    for axis in range(3):
        for value, sgn in ((0.0, -1.0), (1.0, 1.0)):
            T = _cube_boundary_triangles(xyz, tets, axis, value)
            tv = np.array([next((i for i in range(3) if np.linalg.norm(T[e, i] - r) < 1e-12), -1)
                           for e in range(T.shape[0])])
            I = elem.tri_lambda_inv_r(np.repeat(r[None], T.shape[0], 0), T, tv)
            sig = sgn * (T @ A.T + b)[:, :, axis]         # M.n at the triangle vertices
            surf += np.sum(I * sig)
    assert dip == pytest.approx(vol + surf, abs=1e-9 * (abs(dip) + 1))
