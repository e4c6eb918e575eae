"""Write the FP64 oracle's fields at sampled nodes of the full-size workloads.

Full-size meshes are too large for the oracle's complete evaluation inside
a test, so this script (which calls only ``oracle`` and the seeded input
generators) evaluates H_ex, H_ms and H_eff at 4096 seeded random unknowns of
the 1D-periodic wire (about 53k nodes) and of the 3D-periodic composite
(about 1M nodes) and stores them with a hash of the generated inputs:

    python tests/golden/make_expected.py   # -> tests/golden/expected_fullsize.npz
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import model  # noqa: E402
from paper_2409_13958_amd import meshgen as mg  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "expected_fullsize.npz")
SAMPLES = 4096
CHUNK = 256


def input_hash(prob):
    h = hashlib.sha256()
    for a in (prob.xyz, prob.tets, prob.region, prob.m):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def main():
    out = {}
    for name in ("wire_c2", "composite_c3"):
        t = time.time()
        prob = mg.CONFIGS[name]()
        orc = model.Oracle(prob)
        rng = np.random.default_rng(2409139580)
        rows = np.sort(rng.choice(orc.n, size=SAMPLES, replace=False))
        m = orc.unknown_values(prob.m)
        hex_ = orc.heff(m, rows=rows, terms=("ex",))
        # the magnetostatic field row by row is independent of the other rows:
        # evaluate it in blocks of CHUNK rows so that the oracle's per-ring
        # arrays stay within memory, dropping each block's cached operators
        hms = np.empty((rows.size, 3))
        for i0 in range(0, rows.size, CHUNK):
            hms[i0:i0 + CHUNK] = orc.heff(m, rows=rows[i0:i0 + CHUNK], terms=("ms",))
            orc._cache.clear()
            print(f"  {name}: rows {i0 + CHUNK}/{rows.size} ({time.time() - t:.0f} s)",
                  flush=True)
        out[f"{name}_nodes"] = orc.reps[rows]          # representative node of each sample
        out[f"{name}_hex"] = hex_
        out[f"{name}_hms"] = hms
        out[f"{name}_h"] = hex_ + hms
        out[f"{name}_hash"] = np.frombuffer(input_hash(prob).encode(), dtype=np.uint8)
        print(f"{name}: N'={orc.n}, {SAMPLES} samples, {time.time() - t:.0f} s", flush=True)
    np.savez_compressed(OUT, **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
