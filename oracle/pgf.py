"""Periodic Green's function of the Laplacian (paper Sec. 3.2.1, Eq. 2, k0 = 0).

The lattice sums of G0 = 1/|r| in Eq. 2 diverge at zero Bloch phase
(1D logarithmically, 2D linearly, 3D conditionally). The paper evaluates
G^p "via exponentially rapidly convergent sums" without printing them; the
reading used here is the Ewald splitting of 1/r = (2/sqrt(pi)) int_0^inf
exp(-r^2 t^2) dt at t = eta, with Poisson summation of the smooth part over
the periodic axes. Every divergent piece is an additive constant that drops
out because the total charge of a unit cell is zero. Conventions:

* 3D: zero cell average (tin-foil); the k = 0 term is dropped and the
  background constant -pi/(eta^2 V) keeps the result eta-independent.
* 2D (periodic x, y of area A; z normal): keeps the far-field -2 pi |z| / A.
* 1D (period L along one axis; rho = distance from it): keeps the far field
  -(2/L) ln(rho/L) - gamma/L.

``greg0`` is the regular part at the origin, lim_{r->0} (G^p(r) - 1/r), which
carries the interaction of a charge with its own periodic images.

Everything is float64 and vectorised over points; no shortcuts beyond the
formulas. ``lattice_sum`` is the plain brute-force partial sum used to pin
the Ewald forms.
"""
from __future__ import annotations

import numpy as np
from scipy import special

EULER_GAMMA = 0.57721566490153286061
_ERFC_CUT = 6.0      # erfc(6) = 2e-17
_GAUSS_CUT = 6.0     # exp(-k^2/(4 eta^2)) < exp(-36)


def _axes(mask):
    per = [a for a in range(3) if (mask >> a) & 1]
    non = [a for a in range(3) if not (mask >> a) & 1]
    return per, non


def default_eta(mask, L):
    per, _ = _axes(mask)
    Lp = np.array([L[a] for a in per], dtype=np.float64)
    return np.sqrt(np.pi) / np.prod(Lp) ** (1.0 / len(per))


def _reduce(r, mask, L):
    """Shift r by lattice vectors to the minimum image (G^p is periodic)."""
    r = np.array(r, dtype=np.float64, copy=True)
    per, _ = _axes(mask)
    for a in per:
        r[:, a] -= L[a] * np.round(r[:, a] / L[a])
    return r


def _real_space(r, mask, L, eta, skip_origin):
    """sum_n erfc(eta |r + R_n|) / |r + R_n| over the periodic lattice."""
    per, _ = _axes(mask)
    rmax = np.max(np.abs(r), axis=0) if r.shape[0] else np.zeros(3)
    ranges = []
    for a in range(3):
        if a in per:
            nmax = int(np.ceil((_ERFC_CUT / eta + rmax[a]) / L[a])) + 1
            ranges.append(np.arange(-nmax, nmax + 1))
        else:
            ranges.append(np.array([0]))
    out = np.zeros(r.shape[0])
    reach = (_ERFC_CUT + 2.0) / eta + float(np.linalg.norm(rmax))
    for i in ranges[0]:
        for j in ranges[1]:
            for k in ranges[2]:
                R = np.array([i * L[0] if 0 in per else 0.0,
                              j * L[1] if 1 in per else 0.0,
                              k * L[2] if 2 in per else 0.0])
                if np.linalg.norm(R) > reach:
                    continue        # every term of this image is below the cut
                d = np.linalg.norm(r + R, axis=1)
                if skip_origin and i == 0 and j == 0 and k == 0:
                    continue
                with np.errstate(divide="ignore", invalid="ignore"):
                    t = special.erfc(eta * d) / d
                t[eta * d > _ERFC_CUT + 2.0] = 0.0
                out += t
    return out


def _recip_3d(r, L, eta):
    V = L[0] * L[1] * L[2]
    mmax = [int(np.ceil(2 * _GAUSS_CUT * eta * L[a] / (2 * np.pi))) + 1 for a in range(3)]
    out = np.zeros(r.shape[0])
    for i in range(-mmax[0], mmax[0] + 1):
        for j in range(-mmax[1], mmax[1] + 1):
            for k in range(-mmax[2], mmax[2] + 1):
                if i == 0 and j == 0 and k == 0:
                    continue
                kv = 2 * np.pi * np.array([i / L[0], j / L[1], k / L[2]])
                k2 = kv @ kv
                if k2 > (2 * _GAUSS_CUT * eta) ** 2:
                    continue
                out += (4 * np.pi / V) * np.exp(-k2 / (4 * eta * eta)) / k2 * np.cos(r @ kv)
    return out - np.pi / (eta * eta * V)


def _ez_erfc(k, z, eta):
    """exp(k z) erfc(k/(2 eta) + eta z), overflow-free via erfcx."""
    a = k / (2 * eta) + eta * z
    base = -k * k / (4 * eta * eta) - eta * eta * z * z   # k z - a^2
    out = np.where(a >= 0,
                   np.exp(base) * special.erfcx(np.abs(a)),
                   2 * np.exp(k * z) - np.exp(base) * special.erfcx(np.abs(a)))
    return out


def _recip_2d(r, mask, L, eta):
    per, non = _axes(mask)
    a1, a2 = per
    c = non[0]
    A = L[a1] * L[a2]
    z = r[:, c]
    mmax = [int(np.ceil(2 * _GAUSS_CUT * eta * L[a] / (2 * np.pi))) + 1 for a in (a1, a2)]
    out = np.zeros(r.shape[0])
    for i in range(-mmax[0], mmax[0] + 1):
        for j in range(-mmax[1], mmax[1] + 1):
            if i == 0 and j == 0:
                continue
            k1 = 2 * np.pi * i / L[a1]
            k2 = 2 * np.pi * j / L[a2]
            k = np.hypot(k1, k2)
            if k > 2 * _GAUSS_CUT * eta + 0.0:
                continue
            ph = np.cos(k1 * r[:, a1] + k2 * r[:, a2])
            out += (np.pi / A) * ph / k * (_ez_erfc(k, z, eta) + _ez_erfc(k, -z, eta))
    out -= (2 * np.pi / A) * (z * special.erf(eta * z)
                               + np.exp(-eta * eta * z * z) / (eta * np.sqrt(np.pi)))
    return out


def _ein(x):
    """Ein(x) = int_0^x (1 - e^-t)/t dt = E1(x) + gamma + ln x (entire)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    small = x <= 1.0
    xs = x[small]
    term = xs.copy()
    acc = xs.copy()
    for n in range(2, 40):
        term = -term * xs / n
        acc += term / n
    out[small] = acc
    xl = x[~small]
    out[~small] = special.exp1(xl) + EULER_GAMMA + np.log(xl)
    return out


_GL_X, _GL_W = np.polynomial.legendre.leggauss(96)


def _incomplete_k0(k, rho, eta):
    """J(k, rho) = int_0^eta exp(-k^2/(4 t^2) - rho^2 t^2) dt / t."""
    s = 0.5 * (_GL_X + 1.0)              # nodes on (0, 1), t = eta s
    w = 0.5 * _GL_W
    e = np.exp(-k * k / (4 * eta * eta * s[None, :] ** 2)
               - (rho[:, None] * eta * s[None, :]) ** 2) / s[None, :]
    return e @ w


def _recip_1d(r, mask, L, eta):
    per, non = _axes(mask)
    a = per[0]
    Lp = L[a]
    x = r[:, a]
    rho = np.hypot(r[:, non[0]], r[:, non[1]])
    out = np.zeros(r.shape[0])
    mmax = int(np.ceil(2 * _GAUSS_CUT * eta * Lp / (2 * np.pi))) + 1
    for m in range(1, mmax + 1):
        k = 2 * np.pi * m / Lp
        out += (4.0 / Lp) * np.cos(k * x) * _incomplete_k0(k, rho, eta)
    out -= (1.0 / Lp) * (_ein(eta * eta * rho * rho) - np.log(eta * eta * Lp * Lp))
    return out


def pgf(r, mask, L, eta=None):
    """G^p(r) for r [P,3] (metres) away from lattice points; 1/|r| if mask == 0."""
    r = np.atleast_2d(np.asarray(r, dtype=np.float64))
    L = np.asarray(L, dtype=np.float64)
    if mask == 0:
        return 1.0 / np.linalg.norm(r, axis=1)
    if eta is None:
        eta = default_eta(mask, L)
    rr = _reduce(r, mask, L)
    dim = bin(mask).count("1")
    out = _real_space(rr, mask, L, eta, skip_origin=False)
    if dim == 3:
        out += _recip_3d(rr, L, eta)
    elif dim == 2:
        out += _recip_2d(rr, mask, L, eta)
    else:
        out += _recip_1d(rr, mask, L, eta)
    return out


def greg0(mask, L, eta=None):
    """lim_{r->0} [G^p(r) - 1/|r|]: the self-image part of the PGF."""
    L = np.asarray(L, dtype=np.float64)
    if mask == 0:
        return 0.0
    if eta is None:
        eta = default_eta(mask, L)
    z = np.zeros((1, 3))
    dim = bin(mask).count("1")
    val = _real_space(z, mask, L, eta, skip_origin=True)[0] - 2 * eta / np.sqrt(np.pi)
    if dim == 3:
        val += _recip_3d(z, L, eta)[0]
    elif dim == 2:
        val += _recip_2d(z, mask, L, eta)[0]
    else:
        per, _ = _axes(mask)
        Lp = L[per[0]]
        mmax = int(np.ceil(2 * _GAUSS_CUT * eta * Lp / (2 * np.pi))) + 1
        for m in range(1, mmax + 1):
            k = 2 * np.pi * m / Lp
            val += (2.0 / Lp) * special.exp1(k * k / (4 * eta * eta))
        val += np.log(eta * eta * Lp * Lp) / Lp
    return float(val)


def lattice_sum(r, mask, L, radius):
    """Brute-force sum_n 1/|r + R_n| over lattice vectors with |R_n| <= radius
    (a sphere, disc or segment centred on the origin). Diverges with radius;
    only differences between two points are meaningful."""
    r = np.atleast_2d(np.asarray(r, dtype=np.float64))
    per, _ = _axes(mask)
    ranges = []
    for a in range(3):
        if a in per:
            nmax = int(np.floor(radius / L[a]))
            ranges.append(np.arange(-nmax, nmax + 1, dtype=np.float64) * L[a])
        else:
            ranges.append(np.array([0.0]))
    R = np.stack(np.meshgrid(*ranges, indexing="ij"), axis=-1).reshape(-1, 3)
    R = R[np.linalg.norm(R, axis=1) <= radius]
    out = np.zeros(r.shape[0])
    for s in range(0, R.shape[0], 4096):
        d = np.linalg.norm(r[:, None, :] + R[None, s:s + 4096, :], axis=2)
        out += np.sum(1.0 / d, axis=1)
    return out
