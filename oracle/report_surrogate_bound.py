"""What a local surrogate of the grid convolution can reach (test infrastructure).

Step 2 of the AIM (Sec. 3.2.2) convolves the grid charges with the periodic
Green's function sampled on the grid, whose reach is the whole cell. A
network of L convolution layers with 3x3x3 kernels sees only the charges
within L points (per axis) of an output point. Cutting the grid kernel at
that radius, K_R(g) = K(g) for max_a |g_a| <= R and 0 elsewhere, is the
linear operator of that reach closest to K in the coefficients; this script
puts K_R in place of K in the oracle's AIM and reports the relative L2 error
of the magnetostatic field H_ms against the full kernel, for magnetisation
textures of a 2D-periodic film, at several radii R. It calls only the oracle
and the seeded input generators.

    python oracle/report_surrogate_bound.py   # prints one line per texture and radius
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import model  # noqa: E402
from paper_2409_13958_amd import meshgen as mg  # noqa: E402

RADII = (2, 4, 6, 8, 12)


def vortex(L):
    def f(xyz):
        d = xyz[:, :2] - L / 2
        r = np.hypot(d[:, 0], d[:, 1])
        mz = np.exp(-(r / (0.1 * L)) ** 2)
        phi = np.arctan2(d[:, 1], d[:, 0])
        s = np.sqrt(1 - mz * mz)
        return np.stack([-s * np.sin(phi), s * np.cos(phi), mz], axis=1)
    return f


def wall(L):
    def f(xyz):
        mz = np.tanh((xyz[:, 0] - L / 2) / (0.05 * L))
        return np.stack([np.sqrt(1 - mz * mz), np.zeros_like(mz), mz], axis=1)
    return f


def main():
    n, h = 32, 1e-9
    L = n * h
    t0 = time.time()
    textures = {"random": "random", "vortex": vortex(L), "domain wall": wall(L)}
    for name, m in textures.items():
        prob = mg.kuhn_box((n, n, 4), h, periodic=0b011, jitter=0.15, m=m, grid=(n, n, 8))
        orc = model.Oracle(prob)
        mm = orc.unknown_values(prob.m)
        A = orc.aim
        K = A.K.copy()
        ref = orc.heff(mm, method="aim", terms=("ms",))
        idx = [np.arange(s) for s in K.shape]
        dist = [np.minimum(i, s - i) for i, s in zip(idx, K.shape)]
        dmax = np.maximum.reduce(np.meshgrid(*dist, indexing="ij"))
        line = []
        for R in RADII:
            A.Khat = np.fft.fftn(np.where(dmax <= R, K, 0.0))
            got = orc.heff(mm, method="aim", terms=("ms",))
            line.append(f"R={R}: {np.linalg.norm(got - ref) / np.linalg.norm(ref):.2e}")
        A.Khat = np.fft.fftn(K)
        print(f"film {n}x{n}x4 nm, grid {n}x{n}x8, {name}: H_ms rel L2 with the kernel cut at "
              + ", ".join(line) + f" ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
