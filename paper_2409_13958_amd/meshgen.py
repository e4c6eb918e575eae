"""Seeded synthetic inputs: tetrahedral meshes, materials and initial magnetisation.

This module only produces inputs (node coordinates, tetrahedra, region ids,
material constants, periods, grid sizes and unit magnetisation vectors). It
holds none of the field-evaluation arithmetic, so both the FP64 oracle and
the GPU library can be fed from it without sharing any of the method.

The paper's own meshes are not published ("data available on request"), so
every mesh here is synthetic, shaped after the workloads the paper describes:

* ``film_c1``   -- a 2D-periodic thin film (Sec. 4.3 is a film of this kind):
  a structured 10x10x1 hexahedral lattice split into 6 tetrahedra per cube.
* ``wire_c2``   -- a 1D-periodic cylindrical wire (Sec. 4.2): a jittered disk
  triangulation extruded along the periodic axis, prisms split into 3 tets.
* ``composite_c3`` -- a 3D-periodic composite of 27 (possibly overlapping)
  spheres whose parts crossing the cell faces are meshed outside the cell,
  so the unit cell is both touching and protruding (Sec. 2.1, Fig. 1(d)).
* ``kuhn_box``  -- a fully filled, optionally jittered box for small tests.

Meshes that are periodic contain the image nodes on the opposite faces as
separate nodes (touching unit cells); identifying them is left to the code
under test. Random numbers come from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
import numpy as np

SEED0 = 2409139580
NM = 1e-9

# The six tetrahedra of a unit cube along its main diagonal (corner index
# = x + 2y + 4z); each is a monotone lattice path 0 -> 7.
_KUHN = np.array([[0, 1, 3, 7], [0, 1, 5, 7], [0, 2, 3, 7],
                  [0, 2, 6, 7], [0, 4, 5, 7], [0, 4, 6, 7]], dtype=np.int64)
_CORNER = np.array([[(c >> 0) & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)],
                   dtype=np.int64)


@dataclasses.dataclass
class Problem:
    """One synthetic workload: mesh, materials, periodicity, grid, state."""
    name: str
    xyz: np.ndarray          # [N, 3] float64, metres
    tets: np.ndarray         # [T, 4] int32, positive orientation
    region: np.ndarray       # [T] int32
    Ms: np.ndarray           # [R] A/m
    Aex: np.ndarray          # [R] J/m
    periodic: int            # bit0 x, bit1 y, bit2 z
    L: np.ndarray            # [3] metres (ignored on non-periodic axes)
    grid: tuple              # (Nx, Ny, Nz) AIM grid
    m: np.ndarray            # [N, 3] float64 unit vectors, equal on image nodes
    order_p: int = 3
    near_boxes: int = 2
    z0_radius: float = 1.0   # in mean edge lengths

    @property
    def n_nodes(self):
        return self.xyz.shape[0]


def _orient(xyz, tets):
    """Swap two vertices of every negatively oriented tetrahedron."""
    a = xyz[tets[:, 1]] - xyz[tets[:, 0]]
    b = xyz[tets[:, 2]] - xyz[tets[:, 0]]
    c = xyz[tets[:, 3]] - xyz[tets[:, 0]]
    vol = np.einsum("ij,ij->i", a, np.cross(b, c))
    neg = vol < 0
    t = tets.copy()
    t[neg, 2], t[neg, 3] = tets[neg, 3], tets[neg, 2]
    return t, np.abs(vol) / 6.0


def _kuhn_from_cells(cells):
    """Lattice coordinates [6C, 4, 3] of the Kuhn tetrahedra of integer cells [C, 3]."""
    corners = cells[:, None, :] + _CORNER[None, :, :]          # [C, 8, 3]
    return corners[:, _KUHN, :].reshape(-1, 4, 3)                # [6C, 4, 3]


def _unique_nodes(vcoords):
    """Assign node ids to integer lattice coordinates [T, 4, 3]."""
    flat = vcoords.reshape(-1, 3)
    lo = flat.min(axis=0)
    span = flat.max(axis=0) - lo + 1
    key = ((flat[:, 2] - lo[2]) * span[1] + (flat[:, 1] - lo[1])) * span[0] + (flat[:, 0] - lo[0])
    ukey, inv = np.unique(key, return_inverse=True)
    coords = np.empty((ukey.size, 3), dtype=np.int64)
    coords[:, 0] = ukey % span[0] + lo[0]
    coords[:, 1] = (ukey // span[0]) % span[1] + lo[1]
    coords[:, 2] = ukey // (span[0] * span[1]) + lo[2]
    return coords, inv.reshape(-1, 4).astype(np.int32)


def _random_unit(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def kuhn_box(n_cells, h, periodic=0, jitter=0.0, seed=SEED0, Ms=8e5, Aex=1.3e-11,
             grid=None, m="random", name="kuhn_box", region_of=None):
    """A fully filled box of ``n_cells`` cells of side ``h`` (metres; a scalar,
    or three values for boxes), 6 tets each.

    On periodic axes the last node layer is the image of the first and the
    jitter is drawn per wrapped lattice index, so image nodes sit exactly one
    period apart. ``m`` is "random" (iid uniform on the sphere per wrapped
    node) or a callable ``f(xyz) -> [N,3]``. ``region_of`` (optional) maps
    the integer lattice cell of every tetrahedron, an array [T, 3], to its
    region id; ``Ms`` and ``Aex`` then hold one value per region.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = np.asarray(n_cells, dtype=np.int64)
    h = np.asarray(h, dtype=np.float64)
    cells = np.stack(np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]),
                                 indexing="ij"), axis=-1).reshape(-1, 3)
    coords, tets = _unique_nodes(_kuhn_from_cells(cells))
    per = np.array([(periodic >> a) & 1 for a in range(3)], dtype=bool)
    wrap_n = np.where(per, n, n + 1)
    wrapped = coords % wrap_n
    jit = rng.uniform(-jitter, jitter, size=tuple(wrap_n) + (3,))
    xyz = (coords + jit[wrapped[:, 0], wrapped[:, 1], wrapped[:, 2]]) * h
    tets, _ = _orient(xyz, tets)
    L = n * h
    widx = (wrapped[:, 2] * wrap_n[1] + wrapped[:, 1]) * wrap_n[0] + wrapped[:, 0]
    if isinstance(m, str) and m == "random":
        table = _random_unit(rng, int(np.prod(wrap_n)))
        mm = table[widx]
    elif callable(m):
        mm = np.asarray(m(xyz), dtype=np.float64)
    else:
        mm = np.broadcast_to(np.asarray(m, dtype=np.float64), xyz.shape).copy()
    if grid is None:
        grid = tuple(int(max(4, c)) for c in n)
    if region_of is None:
        region = np.zeros(tets.shape[0], np.int32)
    else:
        region = np.asarray(region_of(np.repeat(cells, 6, axis=0)), dtype=np.int32)
    return Problem(name=name, xyz=xyz, tets=tets.astype(np.int32), region=region,
                   Ms=np.atleast_1d(np.asarray(Ms, dtype=np.float64)),
                   Aex=np.atleast_1d(np.asarray(Aex, dtype=np.float64)), periodic=periodic,
                   L=L.astype(np.float64), grid=grid, m=mm)


def ball_regions(n_cells, radius):
    """``region_of`` for kuhn_box: region 1 for the cells whose centre lies
    within ``radius`` cells of the box centre, region 0 elsewhere."""
    ctr = np.asarray(n_cells, dtype=np.float64) / 2.0

    def region_of(cells):
        d = cells + 0.5 - ctr
        return (np.einsum("ij,ij->i", d, d) <= radius * radius).astype(np.int32)
    return region_of


def film_c1(seed=SEED0 + 0):
    """2D-periodic film, 20x20x2 nm, 10x10x1 hexes x 6 tets (242 nodes).

    Periodic in x and y (L = 20 nm), Ms = 8e5 A/m, A = 1.3e-11 J/m, m iid
    uniform on the unit sphere, AIM grid 16x16x4.
    """
    return kuhn_box((10, 10, 1), 2.0 * NM, periodic=0b011, jitter=0.0, seed=seed,
                    Ms=8e5, Aex=1.3e-11, grid=(16, 16, 4), name="film_c1")


def _disk_points(R, s, rng):
    """Jittered triangular lattice inside a disk plus nodes on its circle."""
    nj = int(np.ceil(R / (s * np.sqrt(3) / 2))) + 1
    ni = int(np.ceil(R / s)) + 1
    jj, ii = np.meshgrid(np.arange(-nj, nj + 1), np.arange(-ni, ni + 1), indexing="ij")
    x = (ii + 0.5 * (jj % 2)) * s
    y = jj * s * np.sqrt(3) / 2
    pts = np.stack([x.ravel(), y.ravel()], axis=1)
    pts = pts[np.linalg.norm(pts, axis=1) < R - 0.55 * s]
    pts = pts + rng.uniform(-0.2 * s, 0.2 * s, size=pts.shape)
    nb = int(round(2 * np.pi * R / s))
    ang = (np.arange(nb) + rng.uniform(-0.2, 0.2, size=nb)) * 2 * np.pi / nb
    bnd = R * np.stack([np.cos(ang), np.sin(ang)], axis=1)
    return np.concatenate([pts, bnd], axis=0)


def wire_c2(seed=SEED0 + 1, R=10.0 * NM, period=40.0 * NM, spacing=0.66 * NM,
            n_layers=None, grid=(32, 32, 128), wall_width=8.0 * NM, noise=0.05,
            name="wire_c2"):
    """1D-periodic cylindrical wire along z (radius 10 nm, period 40 nm).

    A jittered disk triangulation (interior lattice jitter +-20 % of the
    spacing, boundary nodes moved only along the circle) is extruded in
    ``n_layers`` flat layers (per-layer z offsets +-20 %), and each prism is
    split into three tetrahedra by the global-index rule so that shared
    quadrilateral faces are cut consistently. Lateral faces stay vertical.
    Ms = 1.4e6 A/m, A = 2e-11 J/m; m is a pair of tanh domain walls along z
    (width 8 nm, exactly periodic) plus 0.05 N(0,1) noise, renormalised.
    """
    from scipy.spatial import Delaunay
    rng = np.random.Generator(np.random.PCG64(seed))
    p2 = _disk_points(R, spacing, rng)
    tri = np.sort(Delaunay(p2).simplices.astype(np.int64), axis=1)
    n2 = p2.shape[0]
    if n_layers is None:
        n_layers = int(round(period / spacing))
    dz = period / n_layers
    zl = (np.arange(n_layers) + rng.uniform(-0.2, 0.2, size=n_layers)) * dz
    zl = np.concatenate([zl, [period + zl[0]]])
    xyz = np.empty(((n_layers + 1) * n2, 3))
    for l in range(n_layers + 1):
        xyz[l * n2:(l + 1) * n2, :2] = p2
        xyz[l * n2:(l + 1) * n2, 2] = zl[l]
    a, b, c = tri[:, 0], tri[:, 1], tri[:, 2]
    blocks = []
    for l in range(n_layers):
        o0, o1 = l * n2, (l + 1) * n2
        blocks.append(np.stack([a + o0, b + o0, c + o0, c + o1], axis=1))
        blocks.append(np.stack([a + o0, b + o0, b + o1, c + o1], axis=1))
        blocks.append(np.stack([a + o0, a + o1, b + o1, c + o1], axis=1))
    tets, _ = _orient(xyz, np.concatenate(blocks, axis=0))
    # magnetisation: generated per wrapped (layer mod n_layers, 2D index)
    noise_tab = rng.standard_normal((n_layers, n2, 3)) * noise
    lay = np.repeat(np.arange(n_layers + 1) % n_layers, n2)
    i2 = np.tile(np.arange(n2), n_layers + 1)
    zw = zl[lay]
    mz = np.tanh(period / (2 * np.pi * wall_width) * np.sin(2 * np.pi * (zw - period / 4) / period))
    mm = np.stack([np.sqrt(np.clip(1 - mz ** 2, 0, None)), np.zeros_like(mz), mz], axis=1)
    mm = mm + noise_tab[lay, i2]
    mm /= np.linalg.norm(mm, axis=1, keepdims=True)
    return Problem(name=name, xyz=xyz, tets=tets.astype(np.int32),
                   region=np.zeros(tets.shape[0], np.int32),
                   Ms=np.array([1.4e6]), Aex=np.array([2e-11]), periodic=0b100,
                   L=np.array([0.0, 0.0, period]), grid=tuple(grid), m=mm)


def gaussian_random_field(xyz, L, corr, rng, kmax_factor=3.0):
    """Periodic smooth unit-vector field: Fourier modes |k| <= 3/corr with
    N(0,1) coefficients damped by exp(-k^2 corr^2 / 4), normalised per node."""
    L = np.asarray(L, dtype=np.float64)
    kmax = kmax_factor / corr
    nmax = np.floor(kmax * L / (2 * np.pi)).astype(int)
    rng_modes = []
    for nx in range(0, nmax[0] + 1):
        for ny in range(-nmax[1], nmax[1] + 1):
            for nz in range(-nmax[2], nmax[2] + 1):
                # one of each +-k pair: the half space nx>0, or nx=0 & ny>0, ...
                if not (nx > 0 or (nx == 0 and (ny > 0 or (ny == 0 and nz > 0)))):
                    continue
                k = 2 * np.pi * np.array([nx, ny, nz]) / L
                if np.dot(k, k) <= kmax * kmax:
                    rng_modes.append((nx, ny, nz))
    modes = np.array(rng_modes, dtype=np.int64)
    kvec = 2 * np.pi * modes / L
    amp = np.exp(-np.sum(kvec ** 2, axis=1) * corr ** 2 / 4)
    coef = rng.standard_normal((modes.shape[0], 3, 2)) * amp[:, None, None]
    out = np.zeros((xyz.shape[0], 3))
    ph = [np.exp(1j * 2 * np.pi * np.outer(xyz[:, a], np.arange(-nmax[a], nmax[a] + 1)) / L[a])
          for a in range(3)]
    chunk = 64
    for s in range(0, modes.shape[0], chunk):
        md = modes[s:s + chunk]
        e = (ph[0][:, md[:, 0] + nmax[0]] * ph[1][:, md[:, 1] + nmax[1]]
             * ph[2][:, md[:, 2] + nmax[2]])                       # [N, c]
        cs = coef[s:s + chunk]
        out += e.real @ cs[:, :, 0] + e.imag @ cs[:, :, 1]
    return out / np.linalg.norm(out, axis=1, keepdims=True)


def composite_c3(seed=SEED0 + 2, period=100.0 * NM, n_cells=144, n_spheres=27,
                 rmin=12.0 * NM, rmax=18.0 * NM, jitter=0.2, grid=(128, 128, 128),
                 corr=10.0 * NM, name="composite_c3"):
    """3D-periodic composite: 27 magnetic spheres in a non-magnetic host.

    A periodic jittered (+-20 %) Kuhn lattice of ``n_cells`` cubes per period
    is cut to the tetrahedra whose centroid lies, in the minimum image, within
    one of the spheres (centres uniform in the cell, radii uniform in
    [12, 18] nm, overlaps allowed). Each kept tetrahedron is placed at the
    periodic image nearest to the centre of the first sphere holding it, so
    spheres crossing a cell face stick out of the cell (protruding) and meet
    their own images there (touching). Only the magnetic host-free part is
    meshed. Material as the film: Ms = 8e5 A/m, A = 1.3e-11 J/m. m is a
    periodic Gaussian random field with correlation length 10 nm.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(n_cells)
    h = period / n
    centres = rng.uniform(0.0, period, size=(n_spheres, 3))
    radii = rng.uniform(rmin, rmax, size=n_spheres)
    jit = rng.uniform(-jitter, jitter, size=(n, n, n, 3))
    # candidate cells: lattice cells whose centre is within (radius + 1.5 h)
    # of a sphere centre in the minimum image; only those are split into tets
    cz = (np.arange(n) + 0.5) * h
    cc = np.stack(np.meshgrid(cz, cz, cz, indexing="ij"), axis=-1).reshape(-1, 3)
    near = np.zeros(cc.shape[0], dtype=bool)
    for s in range(n_spheres):
        d = cc - centres[s]
        d -= np.round(d / period) * period
        near |= np.einsum("ij,ij->i", d, d) <= (radii[s] + 1.5 * h) ** 2
    cand = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n),
                                indexing="ij"), axis=-1).reshape(-1, 3)[near]
    keep_cells, keep_kuhn, keep_shift = [], [], []
    step = 200000
    for c0 in range(0, cand.shape[0], step):
        cells = cand[c0:c0 + step]
        v = _kuhn_from_cells(cells)                                   # [6C,4,3]
        w = v % n
        pos = (v + jit[w[..., 0], w[..., 1], w[..., 2]]) * h
        cen = pos.mean(axis=1)                                        # [6C,3]
        owner = np.full(cen.shape[0], -1, dtype=np.int64)
        shift = np.zeros((cen.shape[0], 3), dtype=np.int64)
        for s in range(n_spheres - 1, -1, -1):
            d = cen - centres[s]
            sh = -np.round(d / period).astype(np.int64)
            dd = d + sh * period
            inside = np.einsum("ij,ij->i", dd, dd) <= radii[s] ** 2
            owner[inside] = s
            shift[inside] = sh[inside]
        sel = owner >= 0
        keep_cells.append(np.repeat(cells, 6, axis=0)[sel])
        keep_kuhn.append(np.tile(np.arange(6), cells.shape[0])[sel])
        keep_shift.append(shift[sel])
    cells = np.concatenate(keep_cells)
    kk = np.concatenate(keep_kuhn)
    shift = np.concatenate(keep_shift)
    corners = cells[:, None, :] + _CORNER[None, :, :]
    v = corners[np.arange(cells.shape[0])[:, None], _KUHN[kk], :] + (shift * n)[:, None, :]
    coords, tets = _unique_nodes(v)
    w = coords % n
    xyz = (coords + jit[w[:, 0], w[:, 1], w[:, 2]]) * h
    tets, _ = _orient(xyz, tets)
    mm = gaussian_random_field(xyz, np.array([period] * 3), corr, rng)
    return Problem(name=name, xyz=xyz, tets=tets.astype(np.int32),
                   region=np.zeros(tets.shape[0], np.int32),
                   Ms=np.array([8e5]), Aex=np.array([1.3e-11]), periodic=0b111,
                   L=np.array([period] * 3), grid=tuple(grid), m=mm)


def _pow2_at_least(v, lo):
    n = lo
    while n < v:
        n *= 2
    return n


def _smooth_at_least(v, lo):
    """Smallest n >= max(v, lo) whose prime factors are 2, 3, 5 and 7."""
    n = max(int(v), int(lo))
    while True:
        k = n
        for f in (2, 3, 5, 7):
            while k % f == 0:
                k //= f
        if k == 1:
            return n
        n += 1


def films_c4(n_films=256, seed=SEED0 + 3, nodes=(5e3, 8e4), period=(20.0 * NM, 200.0 * NM),
             thickness=(2.0 * NM, 10.0 * NM), Ms=(4e5, 1.6e6), Aex=1.3e-11, jitter=0.15,
             extents="smooth"):
    """Independent 2D-periodic films of uneven size (the batched-cell workload).

    Film i: node count log-uniform in ``nodes``, period L uniform in
    ``period`` (square cell, periodic in x and y), thickness t uniform in
    ``thickness``, Ms uniform in ``Ms``; a Kuhn lattice of nx = ny cells of
    side L/nx and nz = t/hz layers (cells as close to cubes as the node count
    allows), jittered; the AIM grid takes the smallest number of points per
    period (at least 16) not coarser than the lattice whose prime factors are
    2, 3, 5 and 7 (``extents="pow2"``: the smallest power of two), and 4 (8
    for five or more layers) across the thickness. The initial state is, in
    turn, a vortex (in-plane curl around the cell centre with an out-of-plane
    core of radius L/10), a uniform tilted state, or iid random directions.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n_films):
        N = float(np.exp(rng.uniform(np.log(nodes[0]), np.log(nodes[1]))))
        L = float(rng.uniform(*period))
        t = float(rng.uniform(*thickness))
        ms = float(rng.uniform(*Ms))
        h = (L * L * t / N) ** (1.0 / 3.0)
        nz = max(1, int(round(t / h)))
        nx = max(4, int(round(np.sqrt(N / (nz + 1)))))
        hxy, hz = L / nx, t / nz
        kind = i % 3
        if kind == 0:
            def mfun(xyz, L=L, t=t):
                d = xyz[:, :2] - L / 2
                r = np.hypot(d[:, 0], d[:, 1])
                mz = np.exp(-(r / (0.1 * L)) ** 2)
                phi = np.arctan2(d[:, 1], d[:, 0])
                sxy = np.sqrt(1 - mz * mz)
                return np.stack([-sxy * np.sin(phi), sxy * np.cos(phi), mz], axis=1)
            m = mfun
        elif kind == 1:
            th, ph = rng.uniform(0.2, 1.4), rng.uniform(0, 2 * np.pi)
            m = [np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)]
        else:
            m = "random"
        nper = _pow2_at_least(nx, 16) if extents == "pow2" else _smooth_at_least(nx, 16)
        grid = (nper, nper, 8 if nz >= 5 else 4)
        out.append(kuhn_box((nx, nx, nz), [hxy, hxy, hz], periodic=0b011, jitter=jitter,
                            seed=seed + 1 + i, Ms=ms, Aex=Aex, grid=grid, m=m,
                            name=f"film_c4_{i}"))
    return out


def film_c5(seed=SEED0 + 4, n_xy=512, n_z=8, grid=None):
    """The surrogate workload: a 2D-periodic film of 512 x 512 x 8 nm on a
    1 nm structured lattice (n_xy x n_xy x n_z cells of 6 tets, 513 x 513 x 9
    node layers, 2.36 M unknowns after the periodic identification), Ms = 8e5
    A/m, A = 1.3e-11 J/m, AIM grid 512 x 512 x 8. ``n_xy`` and ``n_z`` give
    smaller films of the same spacing (grid n_xy x n_xy x n_z by default)."""
    g = grid if grid is not None else (n_xy, n_xy, n_z)
    return kuhn_box((n_xy, n_xy, n_z), 1.0 * NM, periodic=0b011, jitter=0.0, seed=seed,
                    Ms=8e5, Aex=1.3e-11, grid=g, name="film_c5")


CONFIGS = {
    "film_c1": film_c1,
    "wire_c2": wire_c2,
    "composite_c3": composite_c3,
    "film_c5": film_c5,
}
