"""Driver of the continuous-batching SpMV server (spmv_server_* in the C ABI).

Builds a stream of SpMV jobs in pinned host memory, replays one arrival trace
through the server under a policy (0: per-job k-aware auto-tuning, 1: always
CRS), and reports jobs/s and latency percentiles.  A job is a dependent chain
of k SpMVs, y_1 = A x_0 and y_{t+1} = A (2^-shift y_t), the use an iterative
solver makes of a matrix.

    python -m paper_2407_00019_amd.serve [--jobs 2048] [--rate auto] [--slots 4]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from dataclasses import dataclass

import numpy as np
import torch

import paper_2407_00019_amd as spmvat

_HERE = os.path.dirname(os.path.abspath(__file__))

# One slot per hardware queue HIP gives a process by default (four): more
# slots than queues share queues, and a job's chain then waits behind
# another slot's work; measured on MI355X, 4 slots serve about as many jobs
# per second as 8 or 16 slots on 8 or 16 queues.
DEFAULT_SLOTS = 4


@dataclass
class HostJob:
    """One request: CRS with binary32 values, x0, the chain length k and the
    power-of-two scale of the chain, in pinned host memory."""
    id: int
    n: int
    nnz: int
    irp: torch.Tensor
    icol: torch.Tensor
    val: torch.Tensor
    x0: torch.Tensor
    y: torch.Tensor
    k: int
    shift: int
    arrival_s: float
    kind: str = ""

    def descriptor(self, arrival_s: float | None = None) -> spmvat.spmv_job:
        d = spmvat.spmv_job()
        d.id = self.id
        d.arrival_s = self.arrival_s if arrival_s is None else arrival_s
        d.n, d.nnz = self.n, self.nnz
        d.irp, d.icol, d.val = self.irp.data_ptr(), self.icol.data_ptr() if self.nnz else None, \
            self.val.data_ptr() if self.nnz else None
        d.x0, d.y_out = self.x0.data_ptr(), self.y.data_ptr()
        d.k, d.shift = self.k, self.shift
        return d


def chain_shift(n, irp, val32) -> int:
    """Smallest e >= 0 with max_i sum_j |a_ij| <= 2^e, so that the scaled
    chain cannot grow."""
    rows = np.repeat(np.arange(n), np.diff(irp))
    s = np.bincount(rows, weights=np.abs(val32.astype(np.float64)), minlength=n)
    m = float(s.max()) if n else 0.0
    return max(0, int(math.ceil(math.log2(m)))) if m > 1.0 else 0


def pinned(a: np.ndarray) -> torch.Tensor:
    t = torch.empty(a.shape[0], dtype=torch.from_numpy(a[:0]).dtype, pin_memory=True)
    t.numpy()[:] = a
    return t


def build_jobs(specs, seed_x: int = 7) -> list:
    import gen
    jobs = []
    for sp in specs:
        m = sp.matrix()
        v32 = m.val.astype(np.float32)
        x0 = gen.x_uniform(m.n, gen.seed_for(4, 10000 + sp.index)).astype(np.float32)
        jobs.append(HostJob(sp.index, m.n, m.nnz, pinned(m.irp), pinned(m.icol), pinned(v32), pinned(x0),
                            torch.empty(m.n, dtype=torch.float32, pin_memory=True), sp.k,
                            chain_shift(m.n, m.irp, v32), sp.arrival_s, sp.kind))
    return jobs


def load_table(warn=True) -> spmvat.at_table:
    path = os.path.join(_HERE, "at_table.json")
    if not os.path.exists(path):
        return spmvat.at_table_build([], [], None, 1.0)
    with open(path) as f:
        d = json.load(f)
    if warn and spmvat.table_matches_kernels(d) is False:
        print("[serve] warning: at_table.json was measured with other kernel sources "
              "(re-run python -m paper_2407_00019_amd.offline)", file=sys.stderr, flush=True)
    return spmvat.at_table_from_json(d)


def run(jobs, policy: int, slots: int = DEFAULT_SLOTS, hbm_cap: int = 200 << 30, table=None, arrivals=None,
        timeout_s: float = 600.0):
    """Replays the jobs through a fresh server; returns (results, wall_s)."""
    cfg = spmvat.spmv_server_config()
    cfg.slots, cfg.policy, cfg.hbm_cap = slots, policy, hbm_cap
    cfg.table = table if table is not None else load_table()
    srv = spmvat.spmv_server_create(cfg)
    try:
        descs = [j.descriptor(None if arrivals is None else arrivals[i]) for i, j in enumerate(jobs)]
        for d in descs:
            spmvat.spmv_server_submit(srv, d)
        t0 = time.perf_counter()
        spmvat.spmv_server_start(srv)
        st = spmvat.spmv_server_wait(srv, timeout_s)
        wall = time.perf_counter() - t0
        if st != spmvat.SPMV_OK:
            raise RuntimeError("server did not finish in time")
        res = spmvat.spmv_server_results(srv, len(jobs))
    finally:
        spmvat.spmv_server_destroy(srv)
    return res, wall


def summarize(res) -> dict:
    ok = [r for r in res if r.status == spmvat.SPMV_OK]
    lat = np.array([r.done_s - r.arrival_s for r in ok])
    first = min(r.arrival_s for r in res)
    last = max(r.done_s for r in res)
    fmts = {}
    for r in ok:
        name = spmvat.FORMAT_NAMES.get(r.format, str(r.format))
        fmts[name] = fmts.get(name, 0) + 1
    return {"jobs": len(res), "failed": len(res) - len(ok),
            "jobs_per_s": round(len(res) / (last - first), 2) if last > first else None,
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3) if len(lat) else None,
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3) if len(lat) else None,
            "mean_ms": round(float(lat.mean()) * 1e3, 3) if len(lat) else None,
            "span_s": round(last - first, 4), "formats": fmts}


def _median_run(runs, key):
    """The run whose `key` is the median of the runs (runs: list of summaries)."""
    order = sorted(runs, key=lambda r: r[key])
    return order[len(order) // 2]


def compare(jobs_host, slots, hbm_cap, rate, log=print, repeats: int = 3, modes=("burst", "poisson"),
            policies=(("crs", 1), ("auto", 0)), table=None) -> dict:
    """Both policies on one trace, each replayed `repeats` times, alternating
    policies so that drifts of the machine hit both alike: burst first (all
    jobs at t = 0) to find the always-CRS capacity, then Poisson arrivals at
    `rate` jobs/s (rate 'auto': 70% of that capacity).  Each policy reports
    its median run (by jobs/s for the burst, by p50 for Poisson) and every
    run's figure."""
    table = load_table() if table is None else table
    out = {"slots": slots, "hbm_cap_bytes": hbm_cap, "repeats": repeats}
    zeros = [0.0] * len(jobs_host)
    runs = {name: [] for name, _ in policies}
    for rep in range(repeats):
        for name, pol in policies:
            res, wall = run(jobs_host, pol, slots, hbm_cap, table, zeros)
            runs[name].append(summarize(res))
            log(f"[serve] burst {name} #{rep}: {runs[name][-1]}")
    out["burst"] = {name: dict(_median_run(r, "jobs_per_s"), runs_jobs_per_s=[x["jobs_per_s"] for x in r])
                    for name, r in runs.items()}
    if "poisson" not in modes:
        return out
    cap = out["burst"]["crs"]["jobs_per_s"] if "crs" in out["burst"] else list(out["burst"].values())[0]["jobs_per_s"]
    lam = 0.7 * cap if rate == "auto" else float(rate)
    u = np.random.default_rng(20240700019).random(len(jobs_host))
    arr = np.cumsum(-np.log1p(-u) / lam)
    arr -= arr[0]
    runs = {name: [] for name, _ in policies}
    for rep in range(repeats):
        for name, pol in policies:
            res, wall = run(jobs_host, pol, slots, hbm_cap, table, arr.tolist())
            runs[name].append(summarize(res))
            log(f"[serve] poisson {name} #{rep}: {runs[name][-1]}")
    out["poisson"] = {"rate_per_s": round(lam, 2)}
    for name, r in runs.items():
        out["poisson"][name] = dict(_median_run(r, "p50_ms"), runs_p50_ms=[x["p50_ms"] for x in r],
                                    runs_p99_ms=[x["p99_ms"] for x in r])
    return out


def main(argv=None):
    import gen
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=2048)
    ap.add_argument("--slots", type=int, default=DEFAULT_SLOTS)
    ap.add_argument("--cap-gb", type=float, default=200.0)
    ap.add_argument("--rate", default="auto")
    ap.add_argument("--n-max", type=float, default=5e5)
    ap.add_argument("--repeats", type=int, default=3)
    ap.add_argument("--modes", default="burst,poisson", help="burst, poisson or both")
    ap.add_argument("--policies", default="crs,auto", help="crs (always CRS), auto, auto-release (policy 2)")
    ap.add_argument("--kind", default="all", help="all, banded or random: the jobs of one structure only")
    ap.add_argument("--convert-all", action="store_true",
                    help="a table without measured points (D* = +inf): the auto policies convert every job "
                         "whose ELL-Row fits")
    a = ap.parse_args(argv)
    pol_codes = {"crs": 1, "auto": 0, "auto-release": 2}
    policies = tuple((p, pol_codes[p]) for p in a.policies.split(","))
    t0 = time.time()
    specs = gen.serving_jobs(a.jobs, rate_per_s=0.0, n_max=a.n_max)
    if a.kind != "all":
        specs = [sp for sp in specs if sp.kind == a.kind]
    jobs = build_jobs(specs)
    print(f"[serve] built {len(jobs)} jobs ({sum(j.nnz for j in jobs) / 1e6:.1f}M nonzeros) in "
          f"{time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    out = compare(jobs, a.slots, int(a.cap_gb * (1 << 30)), a.rate,
                  log=lambda s: print(s, file=sys.stderr, flush=True), repeats=a.repeats,
                  modes=tuple(a.modes.split(",")), policies=policies,
                  table=spmvat.at_table_build([], [], None, 1.0) if a.convert_all else None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
