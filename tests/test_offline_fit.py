"""The off-line phase's model of the D_mat - R_ell graph (ln R = a + b D over
D <= 1), against exact exponentials and against the measured graph that the
committed table holds."""
import json
import math
import os

import pytest

from paper_2407_00019_amd.offline import fit_rd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_fit_recovers_an_exact_exponential():
    d = [0.0, 0.25, 0.5, 0.75, 1.0, 2.0, 4.0]
    r = [math.exp(0.5 - 3.0 * x) for x in d[:5]] + [123.0, 456.0]   # D > 1 is ignored
    m = fit_rd(d, r)
    assert m["points"] == 5
    assert m["a"] == pytest.approx(0.5, abs=1e-12) and m["b"] == pytest.approx(-3.0, abs=1e-12)
    assert m["rms_ln"] < 1e-12
    assert m["d_cross"] == pytest.approx(0.5 / 3.0, abs=1e-12)
    # another threshold c: the crossing moves to (ln c - a) / b
    assert fit_rd(d, r, c=0.1)["d_cross"] == pytest.approx((math.log(0.1) - 0.5) / -3.0, abs=1e-12)


def test_fit_skips_unmeasured_points_and_needs_a_decreasing_graph():
    d = [0.0, 0.5, 1.0]
    assert fit_rd(d, [2.0, 0.0, 0.5])["points"] == 2              # R = 0 marks an unmeasured point
    assert fit_rd(d, [1.0, 2.0, 4.0])["d_cross"] is None           # rising graph: no crossing
    assert fit_rd([0.0], [1.0]) is None


def test_committed_models_cross_c_inside_the_measured_bracket():
    """For each graph in the committed table, the model's crossing of c lies
    between the last measured point with R >= c and the first with R < c."""
    with open(os.path.join(ROOT, "paper_2407_00019_amd", "at_table.json")) as f:
        t = json.load(f)
    c = t["c"]
    graphs = [k for k in t if k.startswith("graph_vs_")]
    assert graphs
    for key in graphs:
        pts = sorted((p[0], p[1]) for p in t[key] if p[1] > 0)
        first_fail = next(d for d, r in pts if r < c)
        passing = [d for d, r in pts if r >= c and d < first_fail]
        last_pass = max(passing) if passing else -math.inf    # a graph already below c at its first point
        m = t["rd_model" + key[len("graph"):]]
        assert m["rms_ln"] < 0.25, key
        # the fitted line may cross a little before the bracket when the
        # first point sits at c within the timing noise
        assert last_pass < m["d_cross"] <= first_fail + 0.05, (key, last_pass, m["d_cross"], first_fail)
        assert m == fit_rd([p[0] for p in t[key]], [p[1] for p in t[key]], c)


def test_derive_follows_eqs_1_to_3_for_both_crs_kernels():
    """The off-line phase's SP, TT and R_ell (Eqs. (1)-(3)) against the
    oracle's, for both CRS baselines; a point without an ELL-Row measurement
    (refused by the memory guard) gets none."""
    import oracle
    from paper_2407_00019_amd.offline import derive
    p = {"t_crs_scalar": 1.9, "t_crs_best": 0.14, "t_ell": 0.12, "t_trans_ell": 0.29}
    r = derive(p)
    for base in ("scalar", "best"):
        sp = oracle.speedup(p[f"t_crs_{base}"], p["t_ell"])
        tt = oracle.transform_cost(p["t_trans_ell"], p[f"t_crs_{base}"])
        assert r[f"sp_{base}"] == sp and r[f"tt_{base}"] == tt and r[f"r_ell_{base}"] == oracle.r_ell(sp, tt)
    # the worked example under Eq. (3): a 10x speedup bought with a
    # transformation of 10 CRS SpMVs gives R = 1
    r = derive({"t_crs_scalar": 1.0, "t_crs_best": 1.0, "t_ell": 0.1, "t_trans_ell": 10.0})
    assert r["r_ell_best"] == pytest.approx(1.0)
    r = derive({"t_crs_scalar": 1.0, "t_crs_best": 1.0})
    assert r["sp_best"] is None and r["r_ell_scalar"] is None


def test_precision_summary_of_a_two_point_sweep(tmp_path):
    """The per-value-type summary: graph, D* by the table's rule (first D
    whose R falls below c among feasible points), errors and speed-ups."""
    from paper_2407_00019_amd.offline import precision_summary

    def pt(d, r, t_crs, t_ell, err=None, feasible=True):
        q = {"d_mat": d, "r_ell_best": r, "ell_feasible": feasible, "t_crs_best": t_crs, "t_ell": t_ell}
        if err is not None:
            q["rel_l2_vs_f64"] = err
        return q

    sweep = {"sweep": [
        {"family": "local", "f64": pt(0.0, 2.0, 1.0, 0.5), "f32": pt(0.0, 1.5, 0.5, 0.25, 1e-7)},
        {"family": "local", "f64": pt(0.5, 0.8, 1.0, 2.0), "f32": pt(0.5, 1.2, 0.8, 1.0, 2e-7)},
    ]}
    path = tmp_path / "sweep.json"
    path.write_text(json.dumps(sweep))
    s = precision_summary([str(path)])
    f64, f32 = s["families"]["local"]["f64"], s["families"]["local"]["f32"]
    assert f64["d"] == [0.0, 0.5] and f64["r"] == [2.0, 0.8]
    assert f64["d_star"] == pytest.approx(0.5)          # R falls below 1 at D = 0.5
    assert f32["d_star"] == "inf"                       # never below 1
    assert f32["rel_l2_range"] == [1e-7, 2e-7]
    assert f32["speedup_crs_vs_f64"] == [2.0, 1.25]
    assert f32["speedup_ell_vs_f64"] == [2.0, 2.0]
