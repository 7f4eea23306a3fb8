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
