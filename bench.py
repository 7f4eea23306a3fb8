"""Benchmark of the run-time CRS transformation + SpMV hot path on one MI355X.

One step is one pass of the whole path over the 27-point stencil on a 128^3
grid (n = 2,097,152, nnz = 55,742,968, binary64): row statistics and D_mat
(plan creation), the format decision, CRS -> COO-Row, CRS -> CCS,
CCS -> COO-Column, CRS -> ELL-Row, CCS -> ELL-Column, SpMV in every format
and CRS variant, and the reduced-precision rows (values rounded to binary32
and bfloat16, SpMV with binary32 accumulation).  Inputs are resident in HBM
before the timed region; output buffers are allocated once.

Prints ONE JSON line.  `value` is the algorithmic HBM GB/s of the fastest
binary64 SpMV format (bytes the method must move / mean kernel time),
the headline of the metric "SpMV HBM GB/s (% peak) per format"; the
per-format figures, transform cost in CRS-SpMV units (Eq. (2) read as
t_trans / t_crs), SP (Eq. (1)) and R_ell (Eq. (3)) are reported beside it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# the library's column SpMVs privatise y up to this bandwidth (spmvat.h)
def col_paged_max_bw(n):
    return 32192 if n % 4 == 0 else 32576
METRIC = "SpMV HBM GB/s (% peak) per format; transform time / CRS SpMV; jobs/s, p50/p99"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------ algorithmic bytes
# What the method itself must move: each array read or written once, x and
# y once each, ELL padding included (the method computes it).

def stream_lanes(n, nnz):
    """Lanes per row the library's stream CRS kernel picks (its template
    argument, so the kernel's name in a profile): one per 32 entries of the
    mean row, doubled while the grid holds fewer than 1024 workgroups and a
    lane keeps at least four entries."""
    mean = nnz / n if n > 0 else 0.0
    g = 1
    while g < 64 and 32.0 * 2 * g <= mean:
        g *= 2
    while g < 64 and n * g // 256 < 1024 and 4.0 * 2 * g <= mean:
        g *= 2
    return g


def spmv_bytes(fmt, n, nnz, width, vb, xb):
    if fmt == "crs":
        return (vb + 4) * nnz + 4 * (n + 1) + 2 * xb * n
    if fmt in ("coo_row", "coo_col"):
        return (vb + 8) * nnz + 2 * xb * n
    if fmt in ("ell_row", "ell_col"):
        return (vb + 4) * n * width + 2 * xb * n
    raise ValueError(fmt)


def transform_bytes(kind, n, nnz, width, vb):
    if kind == "stats":
        return 4 * (n + 1) + 4 * nnz
    if kind in ("coo_row", "coo_col"):
        return 4 * (n + 1) + 4 * nnz
    if kind == "ccs":
        return (2 * vb + 12) * nnz + 20 * n
    if kind in ("ell_row", "ell_col"):
        return (vb + 4) * nnz + 4 * (n + 1) + (vb + 4) * n * width
    if kind == "convert":
        return 8 * nnz + vb * nnz
    raise ValueError(kind)


# ------------------------------------------------------------- the GPU path

class Timer:
    """HIP events on torch's current stream, the stream every library call
    here is launched on."""

    def __init__(self):
        import torch
        self.torch = torch
        self.marks = {}

    def __call__(self, name, fn, *a, reps=1, **k):
        """Times `reps` back-to-back calls between one pair of events and
        records the mean per call."""
        t = self.torch
        e0, e1 = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            r = fn(*a, **k)
        e1.record()
        self.marks.setdefault(name, []).append((e0, e1, reps))
        return r

    def results_ms(self):
        self.torch.cuda.synchronize()
        return {k: [a.elapsed_time(b) / r for a, b, r in v] for k, v in self.marks.items()}

    def clear(self):
        self.marks = {}


def alloc_like(spmvat, plan, fmt, vt, dev):
    import torch
    s, sz = spmvat.spmv_buffer_sizes(plan, fmt)
    if s != spmvat.SPMV_OK:
        return None, None, sz, s
    vb = torch.empty(0, dtype=vt).element_size()
    if fmt in (spmvat.COO_ROW, spmvat.COO_COL):
        out = [torch.empty(sz.bytes[0] // 4, dtype=torch.int32, device=dev)]
    elif fmt == spmvat.CCS:
        out = [torch.empty(sz.bytes[0] // 4, dtype=torch.int32, device=dev),
               torch.empty(sz.bytes[1] // 4, dtype=torch.int32, device=dev),
               torch.empty(sz.bytes[2] // vb, dtype=vt, device=dev)]
    else:
        out = [torch.empty(sz.bytes[0] // vb, dtype=vt, device=dev),
               torch.empty(sz.bytes[1] // 4, dtype=torch.int32, device=dev)]
    work = torch.empty(max(sz.workspace, 16), dtype=torch.uint8, device=dev)
    return out, work, sz, s


def load_at_table(spmvat):
    path = os.path.join(ROOT, "paper_2407_00019_amd", "at_table.json")
    if os.path.exists(path):
        with open(path) as f:
            return spmvat.at_table_from_json(json.load(f)), path
    return spmvat.at_table_build([], [], None, 1.0), None


class PathRunner:
    """Device buffers for one matrix and one value type, allocated once;
    step() runs the whole path through the C ABI."""

    def __init__(self, spmvat, irp, icol, val, x, label, with_column=True, variants=(0, 1), spmv_reps=3):
        import torch
        self.sp = spmvat
        self.label = label
        self.irp, self.icol, self.val, self.x = irp, icol, val, x
        self.n = irp.numel() - 1
        self.nnz = icol.numel()
        self.dev = irp.device
        self.dtype = spmvat.DTYPE_OF_TORCH[val.dtype]
        self.vt = val.dtype
        self.vb = val.element_size()
        self.xb = x.element_size()
        self.with_column = with_column
        self.variants = variants
        self.reps = spmv_reps
        self.work = torch.empty(spmvat.spmv_plan_workspace_bytes(self.n, self.nnz), dtype=torch.uint8, device=self.dev)
        self.y = torch.empty_like(x)
        # one plan to size the buffers
        plan = spmvat.spmv_plan_create(self.n, self.nnz, irp, icol, val, self.dtype, self.work)
        self.stats = spmvat.spmv_plan_stats(plan)
        # ELL-Row only where the plan's default memory guard admits it (the
        # power-law matrix's would take about 166 GB): then it is reported
        # as refused, as the library refuses it
        st, sz = spmvat.spmv_buffer_sizes(plan, spmvat.ELL_ROW)
        self.ell_row = st == spmvat.SPMV_OK
        self.ell_row_bytes = int(sz.bytes[0] + sz.bytes[1]) if self.ell_row else None
        spmvat.spmv_plan_set_limit(plan, 1 << 45)
        if not self.ell_row:
            s2, sz2 = spmvat.spmv_buffer_sizes(plan, spmvat.ELL_ROW)
            self.ell_row_bytes = int(sz2.bytes[0] + sz2.bytes[1]) if s2 == spmvat.SPMV_OK else None
        self.buf = {}
        fmts = [spmvat.COO_ROW] + ([spmvat.CCS] if with_column else []) + ([spmvat.ELL_ROW] if self.ell_row else [])
        for f in fmts:
            self.buf[f] = alloc_like(spmvat, plan, f, self.vt, self.dev)
        if with_column:
            spmvat.csr_to_ccs(plan, self.buf[spmvat.CCS][0], self.buf[spmvat.CCS][1])
            torch.cuda.synchronize()
            self.stats = spmvat.spmv_plan_stats(plan)
            self.buf[spmvat.COO_COL] = alloc_like(spmvat, plan, spmvat.COO_COL, self.vt, self.dev)
            self.buf[spmvat.ELL_COL] = alloc_like(spmvat, plan, spmvat.ELL_COL, self.vt, self.dev)
        spmvat.spmv_plan_destroy(plan)
        self.ell_w = self.stats.max_row
        self.ellc_w = self.stats.max_col

    def step(self, T, table=None, spmv_only=False):
        sp, L = self.sp, self.label
        plan = T(f"{L}stats", sp.spmv_plan_create, self.n, self.nnz, self.irp, self.icol, self.val, self.dtype,
                 self.work)
        sp.spmv_plan_set_limit(plan, 1 << 45)
        if table is not None:
            self.decision = sp.at_choose_format(plan, table, 0)        # the paper's rule
            self.decision_k100 = sp.at_choose_format(plan, table, 100)  # amortised over 100 SpMVs
        T(f"{L}coo_row", sp.csr_to_coo, plan, 0, self.buf[sp.COO_ROW][0])
        if self.with_column and not spmv_only:
            T(f"{L}ccs", sp.csr_to_ccs, plan, self.buf[sp.CCS][0], self.buf[sp.CCS][1])
            T(f"{L}coo_col", sp.csr_to_coo, plan, 1, self.buf[sp.COO_COL][0])
            T(f"{L}ell_col", sp.csr_to_ell, plan, 1, self.buf[sp.ELL_COL][0])
        if self.ell_row:
            T(f"{L}ell_row", sp.csr_to_ell, plan, 0, self.buf[sp.ELL_ROW][0])
        R = self.reps
        for v in self.variants:
            T(f"{L}spmv_crs{v}", sp.spmv_exec, plan, sp.CRS, v, self.x, self.y, reps=R)
        if self.ell_row:
            T(f"{L}spmv_ell_row", sp.spmv_exec, plan, sp.ELL_ROW, 0, self.x, self.y, reps=R)
        T(f"{L}spmv_coo_row", sp.spmv_exec, plan, sp.COO_ROW, 0, self.x, self.y, reps=R)
        if self.with_column and not spmv_only:
            T(f"{L}spmv_coo_col", sp.spmv_exec, plan, sp.COO_COL, 0, self.x, self.y, reps=R)
            T(f"{L}spmv_ell_col", sp.spmv_exec, plan, sp.ELL_COL, 0, self.x, self.y, reps=R)
            # one atomic add per entry, for comparison with the default kernels
            T(f"{L}spmv_coo_col_atomic", sp.spmv_exec, plan, sp.COO_COL, 1, self.x, self.y, reps=R)
            T(f"{L}spmv_ell_col_atomic", sp.spmv_exec, plan, sp.ELL_COL, 1, self.x, self.y, reps=R)
        sp.spmv_plan_destroy(plan)

    def ccs_algorithms(self, reps=5):
        """Median time (ms) of CRS -> CCS with each algorithm the matrix
        admits, on torch's current stream (the plan built outside the events)."""
        import torch
        sp = self.sp
        out = {}
        for name, alg in (("sort", sp.CCS_SORT), ("bucketed", sp.CCS_BUCKETED), ("banded", sp.CCS_BANDED),
                          ("radix", sp.CCS_RADIX)):
            plan = sp.spmv_plan_create(self.n, self.nnz, self.irp, self.icol, self.val, self.dtype, self.work)
            try:
                sp.spmv_plan_set_ccs_algorithm(plan, alg)
            except sp.SpmvError:
                sp.spmv_plan_destroy(plan)
                continue
            sp.spmv_plan_set_limit(plan, 1 << 45)
            buf, work, _, _ = alloc_like(sp, plan, sp.CCS, self.vt, self.dev)
            ts = []
            for _ in range(reps + 1):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                sp.csr_to_ccs(plan, buf, work)
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            out[name] = round(statistics.median(ts[1:]) * 1e3, 1)
            sp.spmv_plan_destroy(plan)
            del buf, work
        return out

    def release(self):
        """Drops the device buffers (the next workload needs the memory)."""
        self.buf = {}
        self.work = self.y = None

    def outputs(self, fmt, variant=0):
        """y of one format (after the steps), for the error report."""
        sp = self.sp
        plan = sp.spmv_plan_create(self.n, self.nnz, self.irp, self.icol, self.val, self.dtype, self.work)
        sp.spmv_plan_set_limit(plan, 1 << 45)
        if fmt == sp.ELL_ROW:
            sp.csr_to_ell(plan, 0, self.buf[sp.ELL_ROW][0])
        sp.spmv_exec(plan, fmt, variant, self.x, self.y)
        import torch
        torch.cuda.synchronize()
        y = self.y.double().cpu().numpy()
        sp.spmv_plan_destroy(plan)
        return y


def measure(spmvat, m, cfg_index, steps, warmup, spmv_reps, precision, table, log_tag):
    """Times `steps` passes of the whole path over one matrix (after `warmup`
    untimed ones) and derives the per-format rates, transformation costs in
    CRS-SpMV units, SP and R_ell, the format decisions and, for each value
    type in `precision`, the reduced-precision rows."""
    import torch
    import gen
    dev = torch.device("cuda:0")
    x64 = gen.x_uniform(m.n, gen.seed_for(cfg_index))
    irp = torch.from_numpy(m.irp).to(dev)
    icol = torch.from_numpy(m.icol).to(dev)
    val = torch.from_numpy(m.val).to(dev)
    xd = torch.from_numpy(x64).to(dev)
    # lane-group width: the smallest power of two covering half the mean row
    # length (on the 27-point stencil 16 lanes take 223 us, 32 lanes 301 us:
    # a group that is mostly idle lanes keeps fewer rows in flight)
    mu = m.nnz / m.n
    wsub = 2
    while wsub < 64 and wsub < mu / 2:
        wsub *= 2
    v_sub = 1 + int(math.log2(wsub))          # explicit lane-group variant of that width
    runners = [PathRunner(spmvat, irp, icol, val, xd, "", variants=(0, v_sub, 8), spmv_reps=spmv_reps)]
    tags = {spmvat.F32: "f32", spmvat.BF16: "bf16", spmvat.F16: "f16"}
    if precision:
        x32 = xd.float()
        for dt in precision:
            v = spmvat.convert_values(val, dt)
            runners.append(PathRunner(spmvat, irp, icol, v, x32, f"{tags[dt]}:", with_column=False, variants=(8,),
                                      spmv_reps=spmv_reps))
    torch.cuda.synchronize()
    T = Timer()

    def one_step():
        for r in runners:
            r.step(T, table if r.label == "" else None)
        for r, dt in zip(runners[1:], precision):
            T(f"{tags[dt]}:convert", spmvat.spmv_convert_values, val, r.val, dt)

    for _ in range(warmup):
        one_step()
    torch.cuda.synchronize()
    T.clear()
    log(f"[bench] {log_tag}: warmup done ({warmup} steps); timing {steps} steps")
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for _ in range(steps):
        one_step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    raw = T.results_ms()
    ms = {k: statistics.mean(v) for k, v in raw.items()}
    med = {k: statistics.median(v) for k, v in raw.items()}
    ms_per_step = 1000.0 * wall / steps
    log(f"[bench] {log_tag}: timed {steps} steps: {ms_per_step:.3f} ms/step")

    n, nnz = m.n, m.nnz
    r0 = runners[0]
    w, wc = r0.ell_w, r0.ellc_w

    def gbs(b, t_ms):
        return b / (t_ms * 1e-3) / 1e9

    per_format = {}
    spmv_names = {"crs_scalar": ("crs", "spmv_crs0", w), f"crs_subwave{wsub}": ("crs", f"spmv_crs{v_sub}", w),
                  "crs_stream": ("crs", "spmv_crs8", w),
                  "ell_row": ("ell_row", "spmv_ell_row", w), "coo_row": ("coo_row", "spmv_coo_row", w),
                  "coo_col": ("coo_col", "spmv_coo_col", wc), "ell_col": ("ell_col", "spmv_ell_col", wc),
                  "coo_col_atomic": ("coo_col", "spmv_coo_col_atomic", wc),
                  "ell_col_atomic": ("ell_col", "spmv_ell_col_atomic", wc)}
    # rates and ratios from the per-step medians (a host stall between two
    # events inflates one step's mean); "us" keeps the mean
    if not r0.ell_row:
        del spmv_names["ell_row"]
    for name, (fmt, key, width) in spmv_names.items():
        b = spmv_bytes(fmt, n, nnz, width, 8, 8)
        g = gbs(b, med[key])
        per_format[name] = {"us": round(ms[key] * 1e3, 2), "median_us": round(med[key] * 1e3, 2), "gbs": round(g, 1),
                            "frac": round(g / HBM_PEAK_GBS, 4), "bytes": int(b)}
    # the fastest format (a format that moves more bytes per entry would win
    # on GB/s without being faster)
    best = min(per_format, key=lambda k: per_format[k]["median_us"])
    t_crs0 = med["spmv_crs0"]
    t_crs1 = min(med["spmv_crs8"], med[f"spmv_crs{v_sub}"])      # the strong CRS kernel
    transforms = {}
    for kind, width in (("stats", 0), ("coo_row", 0), ("ccs", 0), ("coo_col", 0), ("ell_row", w), ("ell_col", wc)):
        if kind == "ell_row" and not r0.ell_row:
            transforms[kind] = {"refused": "memory guard", "ell_bytes": r0.ell_row_bytes}
            continue
        b = transform_bytes(kind, n, nnz, width, 8)
        transforms[kind] = {"us": round(ms[kind] * 1e3, 2), "median_us": round(med[kind] * 1e3, 2),
                            "gbs": round(gbs(b, med[kind]), 1),
                            "tt_vs_crs_scalar": round(med[kind] / t_crs0, 3),
                            "tt_vs_crs_best": round(med[kind] / t_crs1, 3), "bytes": int(b)}
    sp_ell = r_ell = None
    if r0.ell_row:
        sp_ell = {"vs_crs_scalar": round(t_crs0 / med["spmv_ell_row"], 3),
                  "vs_crs_best": round(t_crs1 / med["spmv_ell_row"], 3)}
        r_ell = {"vs_crs_scalar": round(sp_ell["vs_crs_scalar"] / (med["ell_row"] / t_crs0), 4),
                 "vs_crs_best": round(sp_ell["vs_crs_best"] / (med["ell_row"] / t_crs1), 4)}

    prec = {}
    if precision:
        # reference: this run's binary64 SpMV (the GPU parity tests tie it to the
        # CPU oracle within 1e-13)
        y64 = r0.outputs(spmvat.CRS, 8)
        for r, dt in zip(runners[1:], precision):
            tag, vb = tags[dt], (4 if dt == spmvat.F32 else 2)
            entry = {}
            pairs = [("crs", "spmv_crs8", spmvat.CRS, 8)] + ([("ell_row", "spmv_ell_row", spmvat.ELL_ROW, 0)]
                                                             if r.ell_row else [])
            for fmt, key, code, var in pairs:
                b_ = spmv_bytes(fmt, n, nnz, w, vb, 4)
                t_ms = med[f"{tag}:{key}"]          # median: robust to host stalls between events
                y = r.outputs(code, var)
                err = float(np.linalg.norm(y - y64) / np.linalg.norm(y64))
                entry[fmt if fmt != "crs" else "crs_stream"] = {
                    "mean_us": round(ms[f"{tag}:{key}"] * 1e3, 2), "median_us": round(t_ms * 1e3, 2),
                    "gbs": round(gbs(b_, t_ms), 1), "frac": round(gbs(b_, t_ms) / HBM_PEAK_GBS, 4),
                    "speedup_vs_f64": round(med[key] / t_ms, 3), "rel_l2_vs_f64": float(f"{err:.3e}")}
            entry["convert_us"] = round(ms[f"{tag}:convert"] * 1e3, 2)
            prec[tag] = entry

    if r0.with_column:
        transforms["ccs"]["algorithms_median_us"] = r0.ccs_algorithms()
    decision = {"d_star": table.d_star if math.isfinite(table.d_star) else "inf",
                "choice": spmvat.FORMAT_NAMES[r0.decision[0]] if hasattr(r0, "decision") else None,
                "choice_k100": spmvat.FORMAT_NAMES[r0.decision_k100[0]] if hasattr(r0, "decision_k100") else None}
    if hasattr(r0, "decision_k100"):
        why = r0.decision_k100[2]
        decision["k100_estimates_us"] = {"crs": round(why.t_crs_hat * 1e6, 2), "format": round(why.t_fmt_hat * 1e6, 2),
                                         "transform": round(why.t_trans_hat * 1e6, 2)}
    for r in runners:
        r.release()
    del runners
    return {"m": m, "n": n, "nnz": nnz, "w": w, "wc": wc, "wsub": wsub, "d_mat": r0.stats.d_mat,
            "ms_per_step": ms_per_step,
            "bandwidth": r0.stats.bandwidth,
            "per_format": per_format, "best": best, "transforms": transforms, "sp_ell_row": sp_ell,
            "r_ell_row": r_ell, "precision": prec, "at_decision": decision, "x64": x64, "ell_row": r0.ell_row}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="stencil27_128",
                    choices=["stencil27_128", "laplace64", "powerlaw", "dsweep_d1", "dsweep_local_d1"],
                    help="dsweep_*: the D_mat sweep's matrix at D_mat = 1 (n = 1,048,576, mean 32 per row), "
                         "columns uniform over the row or within 4096 of the diagonal")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-precision", action="store_true", help="skip the reduced-precision rows")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (5-point Laplacian latencies, power-law rows)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the CPU-oracle SpMV sample")
    ap.add_argument("--spmv-reps", type=int, default=3,
                    help="back-to-back SpMVs per format in each step (one event pair around them)")
    ap.add_argument("--serve-repeats", type=int, default=5,
                    help="replays of the serving stream per policy and arrival mode (alternating policies)")
    ap.add_argument("--serve-jobs", type=int, default=2048,
                    help="jobs of the serving stream replayed after the timed steps (0: skip)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run one 1 GiB device copy first (reference kernel for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding this path "
              "over several GPUs is designed but not built", file=sys.stderr)
        sys.exit(2)

    import torch
    import gen
    import paper_2407_00019_amd as spmvat
    if not os.path.exists(spmvat.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()

    dev = torch.device("cuda:0")
    if args.copy_calib:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    builders = {"laplace64": (gen.laplace_64x64, 1), "stencil27_128": (gen.stencil27_128, 2),
                "powerlaw": (gen.powerlaw, 3), "dsweep_d1": (lambda: gen.dsweep_matrix(8), 5),
                "dsweep_local_d1": (lambda: gen.dsweep_matrix(8, local=True), 5)}
    table, table_path = load_at_table(spmvat)
    t0 = time.time()
    build_m, cfg_index = builders[args.workload]
    m = build_m()
    log(f"[bench] workload {m.name}: n={m.n} nnz={m.nnz} generated in {time.time() - t0:.1f}s")
    precision = () if args.no_precision else (spmvat.F32, spmvat.BF16, spmvat.F16)
    h = measure(spmvat, m, cfg_index, args.steps, args.warmup, args.spmv_reps, precision, table, m.name)
    n, nnz, w, best = h["n"], h["nnz"], h["w"], h["best"]
    per_format = h["per_format"]
    head = per_format[best]
    wsub = h["wsub"]
    ell2 = f"k_spmv_ell_row2<double, double, {w if 0 < w <= 32 else 0}>"   # widths 1..32 are unrolled kernels
    wc = h["wc"]
    paged = 0 <= h["bandwidth"] <= col_paged_max_bw(n)   # the column SpMVs' default kernels
    kernel_names = {"ell_row": ell2 if n % 2 == 0 else "k_spmv_ell_row<double, double>",
                    f"crs_subwave{wsub}": f"k_spmv_crs_vector<double, double, {wsub}>",
                    "crs_stream": f"k_spmv_crs_stream<double, double, {stream_lanes(n, nnz)}>",
                    "crs_scalar": "k_spmv_crs_scalar<double, double>", "coo_row": "k_spmv_coo_row<double, double>",
                    "coo_col": "k_spmv_coo_col_pg<double, double>" if paged else "k_spmv_coo_col<double, double>",
                    "ell_col": (("k_spmv_ell_col_pg<double, double, 4, 32768>" if n % 4 == 0
                                 else "k_spmv_ell_col_pg<double, double, 1, 20480>") if paged
                                else "k_spmv_ell_col<double, double>"),
                    "coo_col_atomic": "k_spmv_coo_col<double, double>",
                    "ell_col_atomic": "k_spmv_ell_col<double, double>"}
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        with open(tpath) as f:
            tj = json.load(f)
        # each workload's counters were taken on its own matrix
        section = {"stencil27_128": "kernels", "powerlaw": "powerlaw_kernels", "dsweep_d1": "dsweep_kernels",
                   "dsweep_local_d1": "dsweep_local_kernels"}.get(args.workload)
        ent = tj.get(section, {}).get(kernel_names[best]) if section else None
        if ent and ent.get("source_sha") == kernel_source_sha():
            traffic = ent.get("bytes_per_launch")
    # achieved = algorithmic bytes / mean launch time of the dominant kernel
    achieved = head["bytes"] / (head["us"] * 1e-6) / 1e9
    roofline = {"bound": "hbm", "kernel": kernel_names[best], "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes_per_launch": head["bytes"], "mean_launch_us": head["us"]}
    decision = dict(h["at_decision"])
    decision["table"] = os.path.relpath(table_path, ROOT) if table_path else None
    decision["table_matches_kernels"] = table_matches_kernels(table_path)
    decision.update(model_decision(table_path, h))
    out = {
        "metric": METRIC, "value": roofline["achieved"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(h["ms_per_step"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": m.name, "n": n, "nnz": nnz, "d_mat": h["d_mat"], "ell_width": w,
                   "best_format": best, "headline": f"best-format binary64 SpMV, {m.name}"},
        "roofline": roofline,
        "per_format": per_format,
        "transforms": h["transforms"],
        "sp_ell_row": h["sp_ell_row"], "r_ell_row": h["r_ell_row"],
        "at_decision": decision,
        "precision": h["precision"],
        "kernel_source_sha": kernel_source_sha(),
        "table_kernel_sha": table_kernel_sha(),
    }
    x64 = h.pop("x64")
    if not args.no_extra and args.workload == "stencil27_128":
        extra = {}
        for name, steps in (("laplace64", args.steps), ("powerlaw", max(3, args.steps // 4))):
            build_o, idx_o = builders[name]
            t0 = time.time()
            mo = build_o()
            log(f"[bench] workload {mo.name}: n={mo.n} nnz={mo.nnz} generated in {time.time() - t0:.1f}s")
            ho = measure(spmvat, mo, idx_o, steps, max(1, args.warmup // 2), args.spmv_reps, (), table, mo.name)
            entry = {"workload": mo.name, "n": mo.n, "nnz": mo.nnz, "d_mat": ho["d_mat"], "ell_width": ho["w"],
                     "steps": steps, "ms_per_step": round(ho["ms_per_step"], 3), "at_decision": ho["at_decision"]}
            if name == "laplace64":
                # 0.33 MB: cache-resident and launch-bound, latencies only
                entry["spmv_median_us"] = {k: v["median_us"] for k, v in ho["per_format"].items()}
                entry["transform_median_us"] = {k: v.get("median_us") for k, v in ho["transforms"].items()}
            else:
                entry["per_format"] = ho["per_format"]
                entry["transforms"] = ho["transforms"]
                entry["ell_row"] = "refused by the memory guard" if not ho["ell_row"] else "built"
            extra[name] = entry
            del ho, mo
            torch.cuda.empty_cache()
        out["workloads"] = extra
    if args.serve_jobs > 0:
        out["serving"] = serving(args.serve_jobs, args.serve_repeats)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(m, x64, args.cpu_seconds, with_ell=h["ell_row"])
    print(json.dumps(out), flush=True)


def model_decision(path, h):
    """The paper's rule with D* placed where the fitted D_mat - R_ell model
    of the matrix's locality class crosses c (ELL-Row when D_mat is below
    it and ELL-Row fits), beside this run's measured R_ell against the best
    CRS kernel."""
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        t = json.load(f)
    local = h["bandwidth"] <= 65536
    mdl = t.get("rd_model_vs_best_" + ("local" if local else "scattered")) or {}
    cross = mdl.get("d_cross")
    out = {"d_star_model": cross, "model_class": "local" if local else "scattered"}
    if cross is not None:
        out["choice_model"] = "ell_row" if (h["ell_row"] and h["d_mat"] < cross) else "crs"
    if h.get("r_ell_row"):
        out["r_ell_vs_crs_best_measured"] = h["r_ell_row"]["vs_crs_best"]
    return out


def table_matches_kernels(path):
    """Whether the auto-tuning table was measured with the kernels built here
    (its kernel_source_sha equals the hash of this tree's sources of the
    kernels the off-line phase times), or None without a stamp."""
    if not path or not os.path.exists(path):
        return None
    import paper_2407_00019_amd as spmvat
    with open(path) as f:
        return spmvat.table_matches_kernels(json.load(f))


def serving(count, repeats=5):
    """The serving stream (first `count` jobs), replayed through the
    continuous-batching server, auto-tuned vs always-CRS (binary32)."""
    import gen
    from paper_2407_00019_amd import serve
    t0 = time.time()
    jobs = serve.build_jobs(gen.serving_jobs(count, rate_per_s=0.0))
    log(f"[bench] serving: built {count} jobs ({sum(j.nnz for j in jobs) / 1e6:.0f}M nonzeros) "
        f"in {time.time() - t0:.1f}s")
    res = serve.compare(jobs, slots=serve.DEFAULT_SLOTS, hbm_cap=200 << 30, rate="auto", log=log, repeats=repeats)
    res["jobs_of_stream"] = count
    res["nnz_total"] = int(sum(j.nnz for j in jobs))
    return res


def cpu_model():
    """The host CPU's model name (Linux), for the baseline's record."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def kernel_source_sha():
    from paper_2407_00019_amd import kernel_source_sha as sha
    return sha()


def table_kernel_sha():
    from paper_2407_00019_amd import table_kernel_sha as sha
    return sha()


def cpu_baseline(m, x, budget_s, with_ell=True):
    """The CPU oracle as it stands (single-threaded C, binary64) on the same
    matrix: CRS SpMV repeated for about budget_s seconds; its GB/s uses the
    same algorithmic bytes as the GPU figure."""
    import oracle
    n, nnz = m.n, m.nnz
    times = []
    t_end = time.perf_counter() + budget_s
    while time.perf_counter() < t_end or len(times) < 3:
        t0 = time.perf_counter()
        oracle.spmv_crs(n, m.irp, m.icol, m.val, x)
        times.append(time.perf_counter() - t0)
    t = statistics.median(times)
    b = spmv_bytes("crs", n, nnz, 0, 8, 8)
    # one pass of the oracle's transformations for its own TT figures
    t0 = time.perf_counter(); oracle.csr_to_coo_row(n, m.irp); t_coo = time.perf_counter() - t0
    t_ell = None
    if with_ell:
        t0 = time.perf_counter(); oracle.csr_to_ell_row(n, m.irp, m.icol, m.val); t_ell = time.perf_counter() - t0
    t0 = time.perf_counter(); oracle.csr_to_ccs(n, m.irp, m.icol, m.val); t_ccs = time.perf_counter() - t0
    return {"value": round(b / t / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(times)} CRS SpMVs of {m.name} (median {t * 1e3:.1f} ms each) and one pass of "
                      f"COO-Row / {'ELL-Row / ' if with_ell else ''}CCS transformations",
            "host_cpus": os.cpu_count(), "cpu_model": cpu_model(),
            "tt_coo_row": round(t_coo / t, 3), "tt_ell_row": round(t_ell / t, 3) if t_ell is not None else None,
            "tt_ccs": round(t_ccs / t, 3)}


if __name__ == "__main__":
    main()
