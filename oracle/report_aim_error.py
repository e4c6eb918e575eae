"""AIM error of a full-size workload: the oracle's AIM against its direct sum.

Test infrastructure, like the rest of ``oracle/``: it calls only the oracle
and the seeded input generators. The four-step AIM (Sec. 3.2.2) approximates
the periodic point-charge superposition of Eq. hms_d2; the paper states its
error at the 1e-3 level (Sec. 4). This script measures that error on a
workload that is too large for the direct sum everywhere: at a few seeded
unknowns it evaluates H_ms (and the potential on the rows that H_ms needs,
the samples and their neighbours) once by AIM and once by the direct sum over
all node pairs, and prints the relative L2 error of each. The element-exact
correction u_Z is the same in both and is left in.

    python oracle/report_aim_error.py composite_c3 8 8   # config, samples, processes
    python oracle/report_aim_error.py wire_c2 8 8 3:2,4:2,5:3   # and Lagrange order:near radius pairs

With a list of order:radius pairs the direct sum is computed once and the
AIM (projection, convolution, interpolation and precorrection of that order
and radius) is compared with it for each pair.
"""
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import model  # noqa: E402
from paper_2409_13958_amd import meshgen as mg  # noqa: E402

_ORC = None
_Q = None


def _direct_rows(rows):
    return _ORC._direct(_Q, rows)


def main():
    global _ORC, _Q
    name = sys.argv[1] if len(sys.argv) > 1 else "composite_c3"
    samples = int(sys.argv[2]) if len(sys.argv) > 2 else 8
    procs = int(sys.argv[3]) if len(sys.argv) > 3 else 8
    pairs = [tuple(int(v) for v in s.split(":")) for s in sys.argv[4].split(",")] \
        if len(sys.argv) > 4 else [(None, None)]
    t0 = time.time()
    prob = mg.CONFIGS[name]()
    orc = model.Oracle(prob, order_p=pairs[0][0], near_boxes=pairs[0][1])
    m = orc.unknown_values(prob.m)
    rng = np.random.default_rng(2409139581)
    rows = np.sort(rng.choice(orc.n, size=samples, replace=False))
    ring = orc.ops.neighbours(rows)
    print(f"{name}: N'={orc.n}, {samples} samples, {ring.size} potential rows, "
          f"setup {time.time() - t0:.0f} s", flush=True)
    u_aims = []
    for p, rb in pairs:
        t1 = time.time()
        o = orc if (p, rb) == pairs[0] else model.Oracle(prob, order_p=p, near_boxes=rb)
        u_aims.append(o.potential(m, ring, "aim", z0=False))
        print(f"AIM potential on the rows (p={o.p}, r_b={o.r_b}): "
              f"{time.time() - t1:.0f} s", flush=True)
    _ORC, _Q = orc, orc.charges(m)
    t1 = time.time()
    chunks = np.array_split(ring, max(1, min(procs * 4, ring.size)))
    with Pool(procs) as pool:
        parts = pool.map(_direct_rows, chunks)
    u_dir = np.concatenate(parts)
    print(f"direct potential on the rows: {time.time() - t1:.0f} s ({procs} processes)", flush=True)
    uz = sum(orc.z0(ring)[c] @ m[:, c] for c in range(3))

    def field(u_ring):
        u = np.zeros(orc.n)
        u[ring] = u_ring + uz
        return orc.ops.gradient_field(u, rows)

    h_dir = field(u_dir)

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    for (p, rb), u_aim in zip(pairs, u_aims):
        h_aim = field(u_aim)
        tag = "" if p is None else f"[p={p}, r_b={rb}] "
        print(f"{tag}potential (point charges only) rel L2 AIM vs direct: {rel(u_aim, u_dir):.3e}")
        print(f"{tag}potential (with u_Z) rel L2 AIM vs direct:           "
              f"{rel(u_aim + uz, u_dir + uz):.3e}")
        print(f"{tag}H_ms at the samples rel L2 AIM vs direct:             {rel(h_aim, h_dir):.3e}")
        print(f"{tag}H_ms at the samples max |diff| / max |H_ms|:          "
              f"{float(np.abs(h_aim - h_dir).max() / np.abs(h_dir).max()):.3e}")
    print(f"total {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
