"""Writes gen/dsweep_s.json: the log-sigma s that gives each D_mat target
0, 0.125, ..., 4 for the row-length sweep (n = 1,048,576, mean 32, lengths
clipped to [1, 8192], one shared seeded z vector).

The realised D_mat of a length vector is computed by the CPU oracle only
(Eq. (4)); s is found by bisection.  Run from the repository root:
    python tests/golden/make_dsweep_table.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import gen      # noqa: E402
import oracle   # noqa: E402


def realised(s):
    lens = gen.dsweep_lengths(s)
    irp = np.zeros(lens.shape[0] + 1, np.int64)
    irp[1:] = np.cumsum(lens)
    return oracle.dmat(lens.shape[0], irp.astype(np.int32))


def main():
    out = {"n": gen.DSWEEP_N, "mean": 32.0, "lmin": 1, "lmax": 8192,
           "targets": gen.DSWEEP_TARGETS, "s": [], "realised": []}
    for t in gen.DSWEEP_TARGETS:
        if t == 0:
            s = 0.0
        else:
            lo, hi = 0.0, 4.0
            for _ in range(60):
                mid = 0.5 * (lo + hi)
                if realised(mid) < t:
                    lo = mid
                else:
                    hi = mid
            s = hi
        d = realised(s)
        out["s"].append(s)
        out["realised"].append(d)
        print(f"target {t:6.3f}  s {s:.12f}  realised {d:.6f}", flush=True)
    with open(os.path.join(ROOT, "gen", "dsweep_s.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
