"""Writes gen/table1_s.json: for each matrix of the paper's Table 1
(section 4.2; tests/golden/table1.csv), the lognormal log-sigma s whose
stand-in row lengths (gen.table1_lengths: the printed N and mean, lengths
clipped to [1, 8193] and to a +-4096 column window) have the printed D_mat.

The realised D_mat is computed by the CPU oracle only (Eq. (4)); s is found
by bisection on [0, 4] (the realised D_mat grows with s over that range for
every printed matrix).  Run from the repository root:
    python tests/golden/make_table1_standins.py
"""
import csv
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import gen      # noqa: E402
import oracle   # noqa: E402


def realised(n, mean, s, seed):
    lens = gen.table1_lengths(n, mean, s, seed)
    irp = np.zeros(n + 1, np.int64)
    irp[1:] = np.cumsum(lens)
    return oracle.dmat(n, irp.astype(np.int32)), int(irp[-1])


def main():
    with open(os.path.join(ROOT, "tests", "golden", "table1.csv")) as f:
        rows = list(csv.DictReader(line for line in f if not line.startswith("#")))
    out = {"window": gen.TABLE1_WINDOW, "no": [], "name": [], "n": [], "mu": [], "dmat_printed": [],
           "nnz_printed": [], "s": [], "dmat_realised": [], "nnz_realised": []}
    for r in rows:
        no, n, mu, target = int(r["no"]), int(r["n"]), float(r["mu"]), float(r["dmat"])
        seed = gen.seed_for(6, no)
        lo, hi = 0.0, 4.0
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            if realised(n, mu, mid, seed)[0] < target:
                lo = mid
            else:
                hi = mid
        d, nnz = realised(n, mu, hi, seed)
        for k, v in (("no", no), ("name", r["name"]), ("n", n), ("mu", mu), ("dmat_printed", target),
                     ("nnz_printed", int(r["nnz"])), ("s", hi), ("dmat_realised", d), ("nnz_realised", nnz)):
            out[k].append(v)
        print(f"{no:2d} {r['name']:14s} D {target:5.2f} -> s {hi:.6f} realised {d:.4f}  nnz {nnz} "
              f"(printed {r['nnz']})", flush=True)
    with open(os.path.join(ROOT, "gen", "table1_s.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
