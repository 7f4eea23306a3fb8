"""Off-line phase of the auto-tuner (section 2.2), run once per machine.

For each benchmark matrix (the row-length sweep: n = 1,048,576, mean 32
entries per row, D_mat = 0, 0.125, ..., 4, in two column families: uniform
over the whole row ("scattered") and uniform within 4096 of the diagonal
("local")) it measures on the GPU the CRS
SpMV time t_crs, the ELL-Row SpMV time t_ell and the CRS -> ELL-Row
transformation time t_trans, and computes SP = t_crs / t_ell (Eq. (1)),
TT = t_trans / t_crs (Eq. (2), as the transformation cost in CRS-SpMV units),
R_ell = SP / TT (Eq. (3)) and D_mat (Eq. (4)).  D* is then the smallest D_mat
whose R_ell falls below c = 1 (at_table_build); points where ELL does not
fit the memory limit are recorded as infeasible and left out, as the paper
did for torso1.  The same timings calibrate the cost model used by the
amortised (k-aware) decision: algorithmic bytes per second of each format,
variant and transformation per locality class (bandwidth <= 65536 or not)
and D_mat bucket.

The D_mat - R_ell graph is also modelled (the abstract and section 5 note
that it can be modelled well): ln R_ell = a + b D_mat, fitted by least squares over the
points with D_mat <= 1 (beyond that the longest rows reach the sweep's
8192-entry clip and the graph flattens), with the D_mat where the model
crosses c.

    python -m paper_2407_00019_amd.offline [--points 0,4,8] [--out FILE]
    python -m paper_2407_00019_amd.offline --refit FILE   (models only, no GPU)
    python -m paper_2407_00019_amd.offline --table1 [--out FILE]
    python -m paper_2407_00019_amd.offline --precision-summary SWEEP.json ... --out FILE

--table1 runs the same measurements on stand-ins for the paper's own 22
test matrices (Table 1: the printed N, mean row length and D_mat; see
gen.table1_standin) and writes their D_mat - R_ell graph, D* and model to
table1_standins.json: an off-line phase shaped like the paper's.

Writes at_table.json next to this file by default and prints one JSON line
per point.
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
import torch

import paper_2407_00019_amd as spmvat

_HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(_HERE)


def _bytes(fmt, n, nnz, width, vb, xb):
    if fmt == "crs":
        return (vb + 4) * nnz + 4 * (n + 1) + 2 * xb * n
    if fmt == "coo_row":
        return (vb + 8) * nnz + 2 * xb * n
    if fmt == "ell_row":
        return (vb + 4) * n * width + 2 * xb * n
    raise ValueError(fmt)


def _trans_bytes(fmt, n, nnz, width, vb):
    if fmt == "coo_row":
        return 4 * (n + 1) + 4 * nnz
    if fmt == "ell_row":
        return (vb + 4) * nnz + 4 * (n + 1) + (vb + 4) * n * width
    raise ValueError(fmt)


def time_call(fn, reps=7, warm=2):
    """Median of reps event-timed calls on torch's current stream (ms)."""
    for _ in range(warm):
        fn()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return statistics.median(ts)


def measure_point(m, dtype, x, reps=7, ell_cap=160 << 30):
    """Timings of one matrix in one value type.  Returns a dict (ms)."""
    dev = torch.device("cuda:0")
    irp = torch.from_numpy(m.irp).to(dev)
    icol = torch.from_numpy(m.icol).to(dev)
    val = torch.from_numpy(m.val).to(dev)
    if dtype != spmvat.F64:
        val = spmvat.convert_values(val, dtype)
    xd = x.to(dev) if dtype == spmvat.F64 else x.to(dev).float()
    plan = spmvat.Plan(irp, icol, val)
    st = plan.stats
    n, nnz = m.n, m.nnz
    vb, xb = val.element_size(), xd.element_size()
    y = torch.empty_like(xd)
    out = {"n": n, "nnz": nnz, "d_mat": st.d_mat, "width": st.max_row, "bandwidth": st.bandwidth, "dtype": dtype}
    out["t_crs_scalar"] = time_call(lambda: plan.spmv(spmvat.CRS, xd, y, 0), reps)
    out["t_crs_best"] = time_call(lambda: plan.spmv(spmvat.CRS, xd, y, 1), reps)
    coo_buf = plan._alloc(spmvat.COO_ROW)[0]
    out["t_trans_coo"] = time_call(lambda: spmvat.csr_to_coo(plan.handle, 0, coo_buf), reps)
    out["t_coo"] = time_call(lambda: plan.spmv(spmvat.COO_ROW, xd, y, 0), reps)
    s, sz = plan.sizes(spmvat.ELL_ROW)
    # feasible = within the plan's default memory guard (8x the CRS bytes);
    # the graph is measured beyond it too, up to ell_cap bytes, as the
    # paper's D_mat - R_ell graph covers every matrix that fit its machine
    out["ell_feasible"] = s == spmvat.SPMV_OK
    plan.set_limit(ell_cap)
    s2, sz2 = plan.sizes(spmvat.ELL_ROW)
    out["ell_bytes"] = int(sz2.bytes[0] + sz2.bytes[1])
    y_crs = plan.spmv(spmvat.CRS, xd, None, 1)
    if s2 == spmvat.SPMV_OK:
        ell_buf = plan._alloc(spmvat.ELL_ROW)[0]
        out["t_trans_ell"] = time_call(lambda: spmvat.csr_to_ell(plan.handle, 0, ell_buf), reps)
        out["t_ell"] = time_call(lambda: plan.spmv(spmvat.ELL_ROW, xd, y, 0), reps)
        del ell_buf
    torch.cuda.synchronize()
    out["y"] = y_crs.double().cpu().numpy()
    out["bytes"] = {"crs": _bytes("crs", n, nnz, st.max_row, vb, xb), "coo_row": _bytes("coo_row", n, nnz, 0, vb, xb),
                    "ell_row": _bytes("ell_row", n, nnz, st.max_row, vb, xb),
                    "trans_coo": _trans_bytes("coo_row", n, nnz, 0, vb),
                    "trans_ell": _trans_bytes("ell_row", n, nnz, st.max_row, vb)}
    plan.close()
    torch.cuda.empty_cache()
    return out


def derive(p):
    """Eqs. (1)-(3) against both CRS kernels."""
    r = {}
    for base in ("scalar", "best"):
        t_crs = p[f"t_crs_{base}"]
        if "t_ell" in p:
            sp = t_crs / p["t_ell"]
            tt = p["t_trans_ell"] / t_crs
            r[f"sp_{base}"], r[f"tt_{base}"], r[f"r_ell_{base}"] = sp, tt, sp / tt
        else:
            r[f"sp_{base}"] = r[f"tt_{base}"] = r[f"r_ell_{base}"] = None
    return r


def fit_rd(d, r, c=1.0, dmax=1.0):
    """Least-squares fit of ln R = a + b D over the points with 0 <= D <= dmax
    and R > 0.  Returns a, b, the root-mean-square residual in ln R, the
    number of points used and d_cross = (ln c - a) / b, the D_mat where the
    model's R_ell equals c (None unless b < 0)."""
    pts = [(float(dd), float(rr)) for dd, rr in zip(d, r) if 0.0 <= dd <= dmax and rr > 0.0]
    if len(pts) < 2:
        return None
    x = np.array([p[0] for p in pts])
    y = np.log(np.array([p[1] for p in pts]))
    b, a = np.polyfit(x, y, 1)
    rms = float(np.sqrt(np.mean((y - (a + b * x)) ** 2)))
    cross = (math.log(c) - a) / b if b < 0 else None
    return {"a": float(a), "b": float(b), "rms_ln": rms, "points": len(pts), "d_max": dmax,
            "d_cross": None if cross is None else float(cross)}


def add_rd_models(table):
    """Adds rd_model_vs_{base}_{family} for every stored graph."""
    c = table.get("c", 1.0)
    for key in [k for k in table if k.startswith("graph_vs_")]:
        g = table[key]
        table["rd_model" + key[len("graph"):]] = fit_rd([p[0] for p in g], [p[1] for p in g], c)
    return table


def table1_phase(out_path, c=1.0, reps=7):
    """The off-line phase over the Table 1 stand-ins, binary64."""
    import gen
    tab = gen.table1_recipe()
    rows = []
    for k, no in enumerate(tab["no"]):
        m = gen.table1_standin(no)
        x = torch.from_numpy(gen.x_uniform(m.n, gen.seed_for(6, 200 + no)))
        p = measure_point(m, spmvat.F64, x, reps)
        p.update(derive(p))
        rec = {"no": no, "name": tab["name"][k], "d_printed": tab["dmat_printed"][k],
               "nnz_printed": tab["nnz_printed"][k]}
        rec.update({kk: v for kk, v in p.items() if kk not in ("y", "bytes")})
        rows.append(rec)
        print(json.dumps(rec), flush=True)
    res = {"c": c, "machine": torch.cuda.get_device_name(0), "matrices": rows}
    for base in ("scalar", "best"):
        d = [q["d_mat"] for q in rows]
        r = [q[f"r_ell_{base}"] if q.get(f"r_ell_{base}") else 0.0 for q in rows]
        feas = [1 if q["ell_feasible"] else 0 for q in rows]
        t = spmvat.at_table_build(d, r, feas, c)
        res[f"d_star_vs_{base}"] = t.d_star if math.isfinite(t.d_star) else "inf"
        res[f"graph_vs_{base}"] = [[dd, rr, ff] for dd, rr, ff in zip(d, r, feas)]
        res[f"rd_model_vs_{base}"] = fit_rd(d, r, c)
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1, default=float)
    print(json.dumps({k: v for k, v in res.items() if k.startswith(("d_star", "rd_model"))}), flush=True)


def launch_overhead_s():
    """Time of a CRS SpMV on a tiny matrix: the fixed cost of one launch."""
    import gen
    m = gen.laplace_64x64()
    dev = torch.device("cuda:0")
    plan = spmvat.Plan(torch.from_numpy(m.irp).to(dev), torch.from_numpy(m.icol).to(dev),
                       torch.from_numpy(m.val).to(dev))
    x = torch.ones(m.n, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    t = time_call(lambda: plan.spmv(spmvat.CRS, x, y, 1), 21, 5)
    plan.close()
    return t * 1e-3


def bucket(d):
    """D_mat bucket: how many of the edges 1/16, 1/8, ..., 4 D_mat reaches."""
    return sum(1 for e in spmvat.AT_DBUCKET_EDGES if d >= e)


def locality(bw):
    return 0 if bw <= spmvat.AT_LOCAL_BAND else 1


def model_seconds(cm, fmt, st, k, vb, xb):
    """The cost model's estimate (seconds) of the transformation into fmt plus
    k SpMVs in it, or of k CRS SpMVs (fmt = "crs", the faster CRS variant),
    as the on-line k-aware rule computes it."""
    loc = locality(st.bandwidth)
    b = bucket(st.d_mat)
    n, nnz, w = st.n, st.nnz, st.max_row
    launch = cm["launch_s"]

    def est(bytes_, rate, launches):
        return bytes_ / rate + launches * launch if rate > 0 else math.inf
    if fmt == "crs":
        rates = cm["spmv_bps"][loc][str(spmvat.CRS)]
        return k * min(est(_bytes("crs", n, nnz, w, vb, xb), rates[v][b], 1) for v in (0, 1))
    rate = cm["spmv_bps"][loc][str(spmvat.ELL_ROW)][0][b]
    trate = cm["trans_bps"][loc][str(spmvat.ELL_ROW)][b]
    return est(_trans_bytes("ell_row", n, nnz, w, vb), trate, 1) + k * est(_bytes("ell_row", n, nnz, w, vb, xb), rate, 1)


def calibrate_margin(cm, jobs=96, reps=5, quantile=75.0):
    """The k-aware rule's margin from the model's error on the serving
    stream: for each of the first `jobs` jobs where ELL-Row fits, the ratio
    (transformation + k ELL-Row SpMVs) / (k CRS SpMVs) is predicted by the
    cost model and measured (binary32 values, as the server stores them);
    the margin is exp of the given percentile of |ln(predicted / measured)|,
    so that a conversion is acted on only when its predicted gain exceeds
    the model's usual error."""
    import gen
    dev = torch.device("cuda:0")
    errs = []
    for spec in gen.serving_jobs(jobs, rate_per_s=0.0):
        m = spec.matrix()
        irp = torch.from_numpy(m.irp).to(dev)
        icol = torch.from_numpy(m.icol).to(dev)
        val = torch.from_numpy(m.val).to(dev).float()
        x = torch.from_numpy(gen.x_uniform(m.n, 3)).to(dev).float()
        y = torch.empty_like(x)
        plan = spmvat.Plan(irp, icol, val)
        st = plan.stats
        s, _ = plan.sizes(spmvat.ELL_ROW)
        if s != spmvat.SPMV_OK:
            plan.close()
            continue
        t_crs = time_call(lambda: plan.spmv(spmvat.CRS, x, y, 1), reps) * 1e-3
        ell = plan._alloc(spmvat.ELL_ROW)[0]
        t_tr = time_call(lambda: spmvat.csr_to_ell(plan.handle, 0, ell), reps) * 1e-3
        t_ell = time_call(lambda: plan.spmv(spmvat.ELL_ROW, x, y, 0), reps) * 1e-3
        k = spec.k
        meas = (t_tr + k * t_ell) / (k * t_crs)
        pred = model_seconds(cm, "ell_row", st, k, 4, 4) / model_seconds(cm, "crs", st, k, 4, 4)
        if math.isfinite(pred) and pred > 0:
            errs.append(abs(math.log(pred / meas)))
        plan.close()
        del ell
    torch.cuda.empty_cache()
    if not errs:
        return None
    q = float(np.percentile(errs, quantile))
    return {"k_margin": math.exp(q), "jobs": len(errs), "quantile": quantile,
            "median_abs_ln_err": float(np.median(errs)), "max_abs_ln_err": float(max(errs))}


def precision_summary(paths, c=1.0):
    """From sweeps measured with several value types (the output of this
    module with --dtypes f64,f32,bf16,f16): per column family and value type,
    the D_mat - R_ell graph against the library's CRS kernel, its D* by the
    same rule as the binary64 table, the relative L2 error of y against
    binary64 and the SpMV speed-ups over binary64 (best CRS, ELL-Row)."""
    out = {"c": c, "families": {}}
    for path in paths:
        with open(path) as f:
            sweep = json.load(f)["sweep"]
        for p in sweep:
            fam = out["families"].setdefault(p["family"], {})
            for name in ("f64", "f32", "bf16", "f16"):
                if name not in p:
                    continue
                q, q64 = p[name], p.get("f64", {})
                e = fam.setdefault(name, {"d": [], "r": [], "feasible": [], "rel_l2_vs_f64": [],
                                          "speedup_crs_vs_f64": [], "speedup_ell_vs_f64": []})
                e["d"].append(q["d_mat"])
                e["r"].append(q["r_ell_best"] if "t_ell" in q else 0.0)
                e["feasible"].append(1 if q["ell_feasible"] else 0)
                e["rel_l2_vs_f64"].append(q.get("rel_l2_vs_f64", 0.0))
                e["speedup_crs_vs_f64"].append(q64["t_crs_best"] / q["t_crs_best"] if q64 else 1.0)
                e["speedup_ell_vs_f64"].append(q64["t_ell"] / q["t_ell"] if q64 and "t_ell" in q else None)
    for fam in out["families"].values():
        for e in fam.values():
            t = spmvat.at_table_build(e["d"], e["r"], e["feasible"], c)
            e["d_star"] = t.d_star if math.isfinite(t.d_star) else "inf"
            err = e["rel_l2_vs_f64"]
            e["rel_l2_range"] = [min(err), max(err)]
    return out


def main(argv=None):
    import gen
    ap = argparse.ArgumentParser()
    ap.add_argument("--points", default="all", help="comma-separated sweep indices (0..32) or 'all'")
    ap.add_argument("--dtypes", default="f64,f32,bf16,f16")
    ap.add_argument("--reps", type=int, default=7)
    ap.add_argument("--out", default=os.path.join(_HERE, "at_table.json"))
    ap.add_argument("--c", type=float, default=1.0)
    ap.add_argument("--families", default="scattered,local")
    ap.add_argument("--refit", default=None, help="recompute the D-R models of an existing table and exit")
    ap.add_argument("--table1", action="store_true", help="the off-line phase on the Table 1 stand-ins")
    ap.add_argument("--precision-summary", nargs="+", default=None, metavar="SWEEP",
                    help="summarise sweeps measured with several value types into --out and exit (no GPU)")
    ap.add_argument("--margin-jobs", type=int, default=96,
                    help="serving-stream jobs that calibrate the k-aware margin (0: keep the default)")
    a = ap.parse_args(argv)
    if a.table1:
        out = a.out if a.out != os.path.join(_HERE, "at_table.json") else os.path.join(_HERE, "table1_standins.json")
        table1_phase(out, a.c, a.reps)
        return
    if a.precision_summary:
        if a.out == os.path.join(_HERE, "at_table.json"):
            raise SystemExit("--precision-summary needs its own --out")
        with open(a.out, "w") as f:
            json.dump(precision_summary(a.precision_summary, a.c), f, indent=1, default=float)
        return
    if a.refit:
        with open(a.refit) as f:
            table = add_rd_models(json.load(f))
        with open(a.refit, "w") as f:
            json.dump(table, f, indent=1, default=float)
        print(json.dumps({k: v for k, v in table.items() if k.startswith("rd_model")}), flush=True)
        return
    idx = list(range(len(gen.DSWEEP_TARGETS))) if a.points == "all" else [int(s) for s in a.points.split(",")]
    dts = {"f64": spmvat.F64, "f32": spmvat.F32, "bf16": spmvat.BF16, "f16": spmvat.F16}
    dlist = [dts[s] for s in a.dtypes.split(",")]
    launch_s = launch_overhead_s()
    points = []
    for fam, i in [(f, i) for f in a.families.split(",") for i in idx]:
        t0 = time.time()
        m = gen.dsweep_matrix(i, local=(fam == "local"))
        x = torch.from_numpy(gen.x_uniform(m.n, gen.seed_for(5, 100 + i)))
        res = {}
        for dt in dlist:
            p = measure_point(m, dt, x, a.reps)
            p.update(derive(p))
            res[dt] = p
        y64 = res[spmvat.F64]["y"] if spmvat.F64 in res else None
        rec = {"family": fam, "index": i, "d_target": gen.DSWEEP_TARGETS[i], "gen_s": round(time.time() - t0, 2)}
        for dt, p in res.items():
            name = [k for k, v in dts.items() if v == dt][0]
            q = {k: v for k, v in p.items() if k not in ("y",)}
            if y64 is not None and dt != spmvat.F64:
                q["rel_l2_vs_f64"] = float(np.linalg.norm(p["y"] - y64) / np.linalg.norm(y64))
            rec[name] = q
        points.append(rec)
        print(json.dumps({k: (v if not isinstance(v, dict) else {kk: vv for kk, vv in v.items() if kk != "bytes"})
                          for k, v in rec.items()}), flush=True)

    # the D_mat - R_ell graph in binary64 and D*, against both CRS kernels,
    # per family and over all benchmark points together
    f64 = [p["f64"] for p in points if "f64" in p]
    fams = [p["family"] for p in points if "f64" in p]
    table = {"c": a.c, "machine": torch.cuda.get_device_name(0), "points": len(f64),
             "kernel_source_sha": spmvat.table_kernel_sha()}
    for base in ("scalar", "best"):
        for fam in sorted(set(fams)) + ["all"]:
            sel = [q for q, f in zip(f64, fams) if fam == "all" or f == fam]
            d = [q["d_mat"] for q in sel]
            r = [q[f"r_ell_{base}"] if "t_ell" in q else 0.0 for q in sel]
            feas = [1 if q["ell_feasible"] else 0 for q in sel]
            t = spmvat.at_table_build(d, r, feas, a.c)
            table[f"d_star_vs_{base}_{fam}"] = t.d_star if math.isfinite(t.d_star) else "inf"
            # the same rule over every measured point, memory guard ignored
            meas = [1 if "t_ell" in q else 0 for q in sel]
            t = spmvat.at_table_build(d, r, meas, a.c)
            table[f"d_star_measured_vs_{base}_{fam}"] = t.d_star if math.isfinite(t.d_star) else "inf"
            if fam != "all":
                table[f"graph_vs_{base}_{fam}"] = [[dd, rr, ff] for dd, rr, ff in zip(d, r, feas)]
    # the on-line paper rule falls back to the library's CRS kernel, so D* is
    # taken against it, over every benchmark point
    table["d"] = [q["d_mat"] for q in f64]
    table["r"] = [q["r_ell_best"] if "t_ell" in q else 0.0 for q in f64]
    table["feasible"] = [1 if q["ell_feasible"] else 0 for q in f64]
    # cost model: mean algorithmic bytes/s per locality, format, variant, D bucket
    nb = spmvat.AT_DBUCKETS
    spmv_bps = [{str(f): [[0.0] * nb, [0.0] * nb] for f in (spmvat.CRS, spmvat.COO_ROW, spmvat.ELL_ROW)}
                for _ in range(2)]
    trans_bps = [{str(f): [0.0] * nb for f in (spmvat.COO_ROW, spmvat.ELL_ROW)} for _ in range(2)]
    acc = {}
    for q in f64:
        b, loc = bucket(q["d_mat"]), locality(q["bandwidth"])
        B = q["bytes"]
        obs = [((spmvat.CRS, 0), B["crs"] / (q["t_crs_scalar"] * 1e-3 - launch_s)),
               ((spmvat.CRS, 1), B["crs"] / (q["t_crs_best"] * 1e-3 - launch_s)),
               ((spmvat.COO_ROW, 0), B["coo_row"] / (q["t_coo"] * 1e-3 - 2 * launch_s)),
               (("t", spmvat.COO_ROW), B["trans_coo"] / (q["t_trans_coo"] * 1e-3 - launch_s))]
        if "t_ell" in q:
            obs += [((spmvat.ELL_ROW, 0), B["ell_row"] / (q["t_ell"] * 1e-3 - launch_s)),
                    (("t", spmvat.ELL_ROW), B["trans_ell"] / (q["t_trans_ell"] * 1e-3 - launch_s))]
        for key, v in obs:
            acc.setdefault((loc, key, b), []).append(max(v, 1.0))
    for (loc, key, b), vals in acc.items():
        v = statistics.mean(vals)
        if key[0] == "t":
            trans_bps[loc][str(key[1])][b] = v
        else:
            spmv_bps[loc][str(key[0])][key[1]][b] = v

    # buckets without a sample take the nearest sampled bucket below (else
    # above); a class without any sample for an entry takes the other class's
    def fill(arr):
        for k in range(len(arr)):
            if arr[k] == 0.0:
                lower = [arr[j] for j in range(k - 1, -1, -1) if arr[j] > 0]
                upper = [arr[j] for j in range(k + 1, len(arr)) if arr[j] > 0]
                arr[k] = lower[0] if lower else (upper[0] if upper else 0.0)
    for loc in range(2):
        for f in spmv_bps[loc].values():
            for v in f:
                fill(v)
        for v in trans_bps[loc].values():
            fill(v)
    for loc in range(2):
        other = 1 - loc
        for f, per_v in spmv_bps[loc].items():
            for v_ in range(2):
                if not any(per_v[v_]):
                    per_v[v_] = list(spmv_bps[other][f][v_])
        for f, arr in trans_bps[loc].items():
            if not any(arr):
                trans_bps[loc][f] = list(trans_bps[other][f])
    table["cost_model"] = {"spmv_bps": spmv_bps, "trans_bps": trans_bps, "launch_s": launch_s,
                           "local_band": spmvat.AT_LOCAL_BAND, "d_edges": list(spmvat.AT_DBUCKET_EDGES)}
    add_rd_models(table)
    if a.margin_jobs > 0:
        cal = calibrate_margin(table["cost_model"], a.margin_jobs, max(3, a.reps - 2))
        if cal:
            table["k_margin"] = cal["k_margin"]
            table["k_margin_calibration"] = cal
    table["sweep"] = points
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1, default=float)
    print(json.dumps({k: v for k, v in table.items() if k.startswith(("d_star", "k_margin"))} |
                     {"launch_us": launch_s * 1e6, "out": a.out}), flush=True)


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    main()
