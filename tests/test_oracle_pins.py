"""Pins of the CPU oracle to facts outside itself.

Each test checks the oracle against something it does not compute itself:
dense brute force, Python's stable sort, closed forms, the values printed in
the paper (Table 1, the worked example under Eq. (3)), numpy's own float
conversions and exact rational arithmetic.  A dropped term, a wrong sign or
index, or a transposed operand in the oracle fails at least one of them.
"""
import math
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import gen
import oracle

SMALL_CASES = [
    # (n, seed, max_len, sorted_rows, duplicates, empty_frac)
    (1, 1, 1, True, False, 0.0),
    (7, 2, 4, True, False, 0.3),
    (33, 3, 9, True, False, 0.2),
    (64, 4, 20, True, False, 0.1),
    (40, 5, 6, False, False, 0.2),
    (40, 6, 6, False, True, 0.2),
    (25, 7, 12, True, True, 0.5),
    (16, 8, 0, True, False, 0.0),   # no nonzeros at all
]


def dense_of(n, irp, icol, val):
    a = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(irp))
    np.add.at(a, (rows, icol), val)
    return a


def int_x(n, seed):
    return np.random.default_rng(seed + 100).integers(-3, 4, size=n).astype(np.float64)


@pytest.mark.parametrize("case", SMALL_CASES)
def test_every_format_spmv_equals_dense_product(case):
    """Integer data makes every partial sum exact, so each format's SpMV must
    equal the dense product exactly (a transposed operand or a missed entry
    changes the result)."""
    n, seed, ml, srt, dup, ef = case
    m = gen.random_small(n, seed, ml, srt, dup, ef)
    x = int_x(n, seed)
    yd = dense_of(n, m.irp, m.icol, m.val) @ x
    assert np.array_equal(oracle.spmv_crs(n, m.irp, m.icol, m.val, x), yd)
    irow = oracle.csr_to_coo_row(n, m.irp)
    assert np.array_equal(oracle.spmv_coo_row(n, irow, m.icol, m.val, x), yd)
    ev, ec = oracle.csr_to_ell_row(n, m.irp, m.icol, m.val)
    w = oracle.max_len(n, m.irp)
    assert np.array_equal(oracle.spmv_ell_row(n, w, ev, ec, x), yd)
    ccp, irow_t, val_t = oracle.csr_to_ccs(n, m.irp, m.icol, m.val)
    jcol = oracle.ccs_to_coo_col(n, ccp)
    assert np.array_equal(oracle.spmv_coo_col(n, jcol, irow_t, val_t, x), yd)
    cv, cr = oracle.ccs_to_ell_col(n, ccp, irow_t, val_t)
    wc = oracle.max_len(n, ccp)
    assert np.array_equal(oracle.spmv_ell_col(n, wc, cv, cr, x), yd)


@pytest.mark.parametrize("case", SMALL_CASES)
def test_ccs_is_the_stable_sort_by_column(case):
    """Phase I must place entries in the order of a stable sort of the CRS
    positions by column (Python's sort is stable and shares nothing with the
    counting sort)."""
    n, seed, ml, srt, dup, ef = case
    m = gen.random_small(n, seed, ml, srt, dup, ef, integer_values=False)
    ccp, irow_t, val_t = oracle.csr_to_ccs(n, m.irp, m.icol, m.val)
    rows = np.repeat(np.arange(n), np.diff(m.irp))
    perm = sorted(range(m.nnz), key=lambda p: int(m.icol[p]))
    assert np.array_equal(irow_t, rows[perm].astype(np.int32))
    assert np.array_equal(val_t.view(np.uint64), m.val[perm].view(np.uint64))
    counts = np.bincount(m.icol, minlength=n)
    assert ccp[0] == 0 and ccp[n] == m.nnz
    assert np.array_equal(np.diff(ccp), counts)


def phase1_counting_sort(n, irp, icol, val):
    """The three steps of section 2.1's Phase I in the paper's 1-based
    indexing: count the entries of every column, prefix the counts into the
    column pointer (its last element nnz + 1), then walk the rows in order
    and drop each entry at its column's cursor."""
    IRP = [0] + [int(v) + 1 for v in irp]       # IRP(1..n+1), 1-based
    ICOL = [0] + [int(v) + 1 for v in icol]     # ICOL(1..nnz)
    VAL = [0.0] + [float(v) for v in val]
    nnz = IRP[n + 1] - 1
    cnt = [0] * (n + 2)
    for i in range(1, n + 1):
        for j in range(IRP[i], IRP[i + 1]):
            cnt[ICOL[j]] += 1
    ptr = [0] * (n + 2)
    ptr[1] = 1
    for k in range(2, n + 2):
        ptr[k] = ptr[k - 1] + cnt[k - 1]
    cur = ptr[:]
    irow_t = [0] * (nnz + 1)
    val_t = [0.0] * (nnz + 1)
    for i in range(1, n + 1):
        for j in range(IRP[i], IRP[i + 1]):
            k = cur[ICOL[j]]
            cur[ICOL[j]] = k + 1
            irow_t[k] = i
            val_t[k] = VAL[j]
    return (np.array(ptr[1:], np.int32) - 1, np.array(irow_t[1:], np.int32) - 1,
            np.array(val_t[1:], np.float64))


@pytest.mark.parametrize("case", SMALL_CASES)
def test_ccs_equals_the_papers_counting_sort(case):
    """The oracle builds CCS by sorting (column, position) keys; the paper's
    Phase I builds it by counting and cursor placement.  Both must give the
    same three arrays, bit for bit, also with unsorted rows and duplicates."""
    n, seed, ml, srt, dup, ef = case
    m = gen.random_small(n, seed, ml, srt, dup, ef, integer_values=False)
    ccp, irow_t, val_t = oracle.csr_to_ccs(n, m.irp, m.icol, m.val)
    p_ccp, p_irow, p_val = phase1_counting_sort(n, m.irp, m.icol, m.val)
    assert np.array_equal(ccp, p_ccp)
    assert np.array_equal(irow_t, p_irow)
    assert np.array_equal(val_t.view(np.uint64), p_val.view(np.uint64))


@pytest.mark.parametrize("case", [c for c in SMALL_CASES if not c[4]])
def test_ccs_reads_back_as_the_transpose(case):
    n, seed, ml, srt, dup, ef = case
    m = gen.random_small(n, seed, ml, srt, dup, ef)
    ccp, irow_t, val_t = oracle.csr_to_ccs(n, m.irp, m.icol, m.val)
    assert np.array_equal(dense_of(n, ccp, irow_t, val_t), dense_of(n, m.irp, m.icol, m.val).T)


@pytest.mark.parametrize("case", SMALL_CASES)
def test_crs_ccs_crs_round_trip(case):
    """Applying Phase I twice returns the input when rows are sorted, and the
    row-sorted input (stable within a row) otherwise."""
    n, seed, ml, srt, dup, ef = case
    m = gen.random_small(n, seed, ml, srt, dup, ef, integer_values=False)
    ccp, irow_t, val_t = oracle.csr_to_ccs(n, m.irp, m.icol, m.val)
    irp2, icol2, val2 = oracle.csr_to_ccs(n, ccp, irow_t, val_t)
    assert np.array_equal(irp2, m.irp)
    want_c, want_v = m.icol.copy(), m.val.copy()
    for i in range(n):
        a, b = m.irp[i], m.irp[i + 1]
        o = np.argsort(m.icol[a:b], kind="stable")
        want_c[a:b] = m.icol[a:b][o]
        want_v[a:b] = m.val[a:b][o]
    assert np.array_equal(icol2, want_c)
    assert np.array_equal(val2.view(np.uint64), want_v.view(np.uint64))
    if srt:
        assert np.array_equal(icol2, m.icol)


@pytest.mark.parametrize("case", SMALL_CASES)
def test_coo_row_invariants(case):
    n, seed, ml, srt, dup, ef = case
    m = gen.random_small(n, seed, ml, srt, dup, ef)
    irow = oracle.csr_to_coo_row(n, m.irp)
    assert irow.shape[0] == m.nnz
    assert np.all(np.diff(irow) >= 0)
    assert np.array_equal(np.bincount(irow, minlength=n), np.diff(m.irp))
    a = np.zeros((n, n))
    np.add.at(a, (irow, m.icol), m.val)
    assert np.array_equal(a, dense_of(n, m.irp, m.icol, m.val))


@pytest.mark.parametrize("case", SMALL_CASES)
def test_ell_invariants(case):
    """ELL width = longest row; padding is +0.0 (all bits zero) with the
    row's own index; the first l_i slots of row i are the CRS row in order;
    the non-padding count is nnz."""
    n, seed, ml, srt, dup, ef = case
    m = gen.random_small(n, seed, ml, srt, dup, ef, integer_values=False)
    lens = np.diff(m.irp)
    w = int(lens.max()) if n else 0
    assert oracle.max_len(n, m.irp) == w
    ev, ec = oracle.csr_to_ell_row(n, m.irp, m.icol, m.val)
    assert ev.shape[0] == w * n
    ev2, ec2 = ev.reshape(w, n), ec.reshape(w, n)      # [slot, row]
    real = np.arange(w)[:, None] < lens[None, :]
    assert int(real.sum()) == m.nnz
    assert np.all(ev2[~real].view(np.uint64) == 0)
    assert np.all(ec2[~real] == np.broadcast_to(np.arange(n), (w, n))[~real])
    for i in range(n):
        a, b = m.irp[i], m.irp[i + 1]
        assert np.array_equal(ev2[: b - a, i].view(np.uint64), m.val[a:b].view(np.uint64))
        assert np.array_equal(ec2[: b - a, i], m.icol[a:b])


@pytest.mark.parametrize("case", SMALL_CASES)
def test_ell_col_invariants(case):
    n, seed, ml, srt, dup, ef = case
    m = gen.random_small(n, seed, ml, srt, dup, ef)
    ccp, irow_t, val_t = oracle.csr_to_ccs(n, m.irp, m.icol, m.val)
    counts = np.bincount(m.icol, minlength=n)
    w = int(counts.max()) if m.nnz else 0
    cv, cr = oracle.ccs_to_ell_col(n, ccp, irow_t, val_t)
    assert cv.shape[0] == w * n
    cv2, cr2 = cv.reshape(w, n), cr.reshape(w, n)
    real = np.arange(w)[:, None] < counts[None, :]
    assert np.all(cv2[~real].view(np.uint64) == 0)
    assert np.all(cr2[~real] == np.broadcast_to(np.arange(n), (w, n))[~real])
    a = np.zeros((n, n))
    cols = np.broadcast_to(np.arange(n), (w, n))
    np.add.at(a, (cr2[real], cols[real]), cv2[real])
    assert np.array_equal(a, dense_of(n, m.irp, m.icol, m.val))


def test_all_formats_give_one_exact_order_result():
    """For sorted, duplicate-free rows the five loop orders add each row's
    products in the same order, so the binary64 results agree bit for bit
    (up to the sign of zero) even with non-integer data."""
    m = gen.lognormal_matrix(3000, 12.0, 0.8, 77, 1, 200)
    x = gen.x_uniform(m.n, 78)
    n = m.n
    y = oracle.spmv_crs(n, m.irp, m.icol, m.val, x)
    irow = oracle.csr_to_coo_row(n, m.irp)
    ev, ec = oracle.csr_to_ell_row(n, m.irp, m.icol, m.val)
    ccp, irow_t, val_t = oracle.csr_to_ccs(n, m.irp, m.icol, m.val)
    cv, cr = oracle.ccs_to_ell_col(n, ccp, irow_t, val_t)
    outs = [
        oracle.spmv_coo_row(n, irow, m.icol, m.val, x),
        oracle.spmv_ell_row(n, oracle.max_len(n, m.irp), ev, ec, x),
        oracle.spmv_coo_col(n, oracle.ccs_to_coo_col(n, ccp), irow_t, val_t, x),
        oracle.spmv_ell_col(n, oracle.max_len(n, ccp), cv, cr, x),
    ]
    for o in outs:
        assert np.array_equal(o, y)
    # and the result is not the transpose product
    assert not np.allclose(y, dense_of(n, m.irp, m.icol, m.val).T @ x)


# ------------------------------------------------------------- D_mat, Eq. (4)

def exact_dmat(counts_by_len):
    """D_mat = sigma/mu from a {length: rows} histogram, to 40 digits."""
    n = sum(counts_by_len.values())
    s1 = sum(l * c for l, c in counts_by_len.items())
    s2 = sum(l * l * c for l, c in counts_by_len.items())
    getcontext().prec = 50
    num = Decimal(n * s2 - s1 * s1)
    return n, s1, s2, float(num.sqrt() / Decimal(s1)) if s1 else 0.0


def test_dmat_laplace_64_closed_form():
    # 5-point grid 64x64: 4 corner rows of 3, 248 edge rows of 4, 3844 interior rows of 5
    n, s1, s2, d = exact_dmat({3: 4, 4: 4 * 62, 5: 62 * 62})
    m = gen.laplace_64x64()
    assert oracle.row_moments(m.n, m.irp) == (s1, s2, 5, 3)
    mu, sg, dd = oracle.dmat_from_moments(n, s1, s2)
    assert mu == 20224 / 4096
    assert dd == pytest.approx(d, rel=2e-16, abs=0)
    assert round(dd, 7) == 0.0498355


def stencil27_lengths(edge):
    """{length: rows} of the 27-point stencil with Dirichlet truncation: a row
    with a boundary coordinate on `a` of the three axes has 3^(3-a) 2^a
    entries."""
    inner = edge - 2
    return {27: inner ** 3, 18: 3 * 2 * inner ** 2, 12: 3 * 4 * inner, 8: 8}


def test_dmat_stencil27_closed_form_small():
    n, s1, s2, d = exact_dmat(stencil27_lengths(12))
    m = gen.stencil27(12, 12, 12, 1)
    assert m.nnz == (3 * 10 + 4) ** 3
    assert oracle.row_moments(m.n, m.irp) == (s1, s2, 27, 8)
    assert oracle.dmat(m.n, m.irp) == pytest.approx(d, rel=2e-16, abs=0)


@pytest.mark.slow
def test_dmat_stencil27_128_closed_form():
    n, s1, s2, d = exact_dmat(stencil27_lengths(128))
    assert s1 == 382 ** 3 == 55_742_968
    m = gen.stencil27_128()
    assert oracle.row_moments(m.n, m.irp) == (s1, s2, 27, 8)
    dd = oracle.dmat(m.n, m.irp)
    assert dd == pytest.approx(d, rel=2e-16, abs=0)
    assert round(dd, 7) == 0.0720398


@pytest.mark.parametrize("a,b,rows", [(1, 3, 10), (5, 9, 1000), (0, 7, 6), (32, 8192, 4)])
def test_dmat_two_valued_rows(a, b, rows):
    """Half the rows of length a, half of length b: sigma = |a-b|/2,
    mu = (a+b)/2, so D_mat = |a-b|/(a+b)."""
    lens = np.array([a, b] * rows, np.int32)
    irp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    d = oracle.dmat(lens.shape[0], irp)
    assert d == pytest.approx(abs(a - b) / (a + b), rel=1e-15)


def test_dmat_constant_rows_and_empty():
    irp = np.arange(0, 11 * 7, 7, dtype=np.int32)
    assert oracle.dmat(10, irp) == 0.0
    assert oracle.dmat(5, np.zeros(6, np.int32)) == 0.0
    assert oracle.dmat(1, np.array([0, 3], np.int32)) == 0.0


@pytest.mark.parametrize("case", SMALL_CASES)
def test_bandwidth_is_max_distance_over_entries(case):
    n, seed, ml, srt, dup, ef = case
    m = gen.random_small(n, seed, ml, srt, dup, ef)
    rows = np.repeat(np.arange(n), np.diff(m.irp))
    want = int(np.abs(rows - m.icol).max()) if m.nnz else 0
    assert oracle.bandwidth(n, m.irp, m.icol) == want


def test_bandwidth_of_stencils_and_windows():
    m = gen.laplace_64x64()
    assert oracle.bandwidth(m.n, m.irp, m.icol) == 64
    m = gen.stencil27(10, 10, 10, 1)
    assert oracle.bandwidth(m.n, m.irp, m.icol) == 1 + 10 + 100
    lens = np.full(5000, 7, np.int32)
    m = gen.window_rows(5000, lens, 40, 3)
    assert oracle.bandwidth(m.n, m.irp, m.icol) <= 40
    # an arrow matrix (dense first row and column): bandwidth n - 1, whatever
    # the order of the entries inside the rows
    n = 300
    rows = [[0] + list(range(n - 1, 0, -1))] + [[i, 0] for i in range(1, n)]
    irp = np.cumsum([0] + [len(r) for r in rows]).astype(np.int32)
    icol = np.concatenate([np.array(r, np.int32) for r in rows])
    assert oracle.bandwidth(n, irp, icol) == n - 1
    # a diagonal matrix has bandwidth 0, an empty one too
    assert oracle.bandwidth(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32)) == 0
    assert oracle.bandwidth(n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32)) == 0


def test_u128_rounding_matches_python():
    """Python's int -> float is correctly rounded (ties to even)."""
    rng = np.random.default_rng(5)
    vals = [0, 1, (1 << 53) + 1, (1 << 54) + 2, (1 << 54) + 6, (1 << 127) - 1, 3 << 70]
    vals += [int(rng.integers(0, 1 << 62)) * int(rng.integers(0, 1 << 62)) for _ in range(2000)]
    for v in vals:
        assert oracle.u128_to_double(v) == float(v)


def trunc2(v):
    return math.floor(v * 100 + 1e-9) / 100


def test_table1_dmat_is_sigma_over_mu():
    """Table 1 prints N, NNZ, mu, sigma and D_mat truncated to two decimals.
    Feeding the oracle moments with that N, NNZ and a sigma inside the
    printed truncation interval must reproduce the printed D_mat for all 22
    matrices (mu/sigma, sigma^2/mu or a dropped term would not)."""
    import csv
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "table1.csv")
    rows = [r for r in csv.DictReader(l for l in open(path) if not l.startswith("#"))]
    assert len(rows) == 22
    mu_ok = 0
    for r in rows:
        n, nnz = int(r["n"]), int(r["nnz"])
        sig, dprint = float(r["sigma"]), float(r["dmat"])
        if trunc2(nnz / n) == float(r["mu"]):
            mu_ok += 1
        hits = []
        for s in np.linspace(sig, sig + 0.00999, 12):
            s2 = round((n * n * s * s + nnz * nnz) / n)
            mu, sg, d = oracle.dmat_from_moments(n, nnz, s2)
            hits.append(trunc2(d) == dprint)
        assert any(hits), r["name"]
    # the mean column agrees with NNZ/N except the torso2 misprint
    assert mu_ok == 21


# ----------------------------------------------------------- Eqs. (1)-(3), D*

def test_worked_example_under_eq3():
    """A 10x ELL speedup with a transformation costing 10 CRS SpMVs gives
    R_ell = 1.0 (section 2.2, text after Eq. (3))."""
    t_crs, t_ell, t_trans = 1.0, 0.1, 10.0
    sp = oracle.speedup(t_crs, t_ell)
    tt = oracle.transform_cost(t_trans, t_crs)
    assert sp == pytest.approx(10.0)
    assert tt == pytest.approx(10.0)
    assert oracle.r_ell(sp, tt) == pytest.approx(1.0)


def test_dstar_rule():
    inf = math.inf
    # monotone: R falls below c = 1 first at D = 0.5
    pts = [(0.1, 5.0, True), (0.3, 1.5, True), (0.5, 0.9, True), (0.8, 0.2, True)]
    assert oracle.d_star(pts) == 0.5
    # all profitable / none profitable
    assert oracle.d_star([(0.1, 2.0, True), (3.1, 1.0, True)]) == inf
    assert oracle.d_star([(0.02, 0.5, True), (1.0, 0.1, True)]) == 0.02
    # non-monotone: the first failure decides
    assert oracle.d_star([(0.1, 2, True), (0.2, 0.5, True), (0.4, 3, True)]) == 0.2
    # infeasible points (ELL did not fit) are left out
    assert oracle.d_star([(0.1, 2, True), (5.72, 0.0, False)]) == inf
    # a tie at equal D with one failure counts as failure there
    assert oracle.d_star([(0.3, 2, True), (0.3, 0.5, True)]) == 0.3
    assert oracle.choose_paper(0.29, 0.3) == "ell_row"
    assert oracle.choose_paper(0.3, 0.3) == "crs"
    assert oracle.choose_paper(7.0, inf) == "ell_row"


def test_k_aware_break_even():
    """Converting pays after k SpMVs iff t_trans + k t_f < k t_crs, i.e.
    k > TT / (1 - 1/SP)."""
    t_crs, t_f, t_tr = 1.0, 0.5, 3.0        # SP = 2, TT = 3: break-even k = 6
    assert oracle.choose_k_aware(5, t_crs, {"ell_row": (t_tr, t_f)}) == "crs"
    assert oracle.choose_k_aware(6, t_crs, {"ell_row": (t_tr, t_f)}) == "crs"   # tie
    assert oracle.choose_k_aware(7, t_crs, {"ell_row": (t_tr, t_f)}) == "ell_row"
    both = {"ell_row": (3.0, 0.5), "coo_row": (0.2, 0.9)}
    assert oracle.choose_k_aware(1, t_crs, both) == "crs"
    assert oracle.choose_k_aware(3, t_crs, both) == "coo_row"
    assert oracle.choose_k_aware(100, t_crs, both) == "ell_row"
    # with a margin m the break-even moves to k > m TT / (1 - m/SP):
    # m = 1.1 gives k > 3.3 / 0.45 = 7.33
    assert oracle.choose_k_aware(7, t_crs, {"ell_row": (t_tr, t_f)}, 1.1) == "crs"
    assert oracle.choose_k_aware(8, t_crs, {"ell_row": (t_tr, t_f)}, 1.1) == "ell_row"
    # a format less than m times faster never pays, whatever k
    assert oracle.choose_k_aware(10**9, t_crs, {"ell_row": (0.0, 0.95)}, 1.1) == "crs"


# ------------------------------------------------------ value rounding (RNE)

def _format_table(dtype):
    if dtype == oracle.BF16:
        pats = np.arange(0, 0x7F80, dtype=np.uint32)
        vals = (pats << 16).view(np.float32).astype(np.float64)
    else:
        pats = np.arange(0, 0x7C00, dtype=np.uint16)
        vals = pats.view(np.float16).astype(np.float64)
    return pats.astype(np.int64), vals


def brute_round(v, pats, vals):
    """Nearest format value by exact rational distance over the format's own
    finite non-negative values; ties to the even bit pattern; overflow to
    inf when |v| reaches max + half a step."""
    a = abs(v)
    sign = 0x8000 if math.copysign(1.0, v) < 0 else 0
    top = Fraction(vals[-1]) + (Fraction(vals[-1]) - Fraction(vals[-2])) / 2
    if Fraction(a) >= top:
        return sign | (0x7F80 if vals.shape[0] == 0x7F80 else 0x7C00)
    i = int(np.searchsorted(vals, a))
    cands = [j for j in (i - 1, i) if 0 <= j < vals.shape[0]]
    best = None
    for j in cands:
        dist = abs(Fraction(a) - Fraction(float(vals[j])))
        key = (dist, int(pats[j]) & 1)
        if best is None or key < best[0]:
            best = (key, j)
    return sign | int(pats[best[1]])


def _probe_values(rng, lo_exp, hi_exp, pats, vals):
    out = []
    e = rng.integers(lo_exp, hi_exp, size=300)
    out += list(rng.uniform(1, 2, size=300) * np.exp2(e.astype(np.float64)) * rng.choice([-1, 1], 300))
    # exact midpoints between neighbours, and one binary64 step either side
    idx = rng.integers(1, vals.shape[0] - 1, size=200)
    for j in idx:
        mid = (vals[j] + vals[j + 1]) / 2
        out += [mid, np.nextafter(mid, np.inf), np.nextafter(mid, -np.inf), -mid]
    out += [0.0, -0.0, float(vals[1]) / 2, float(vals[1]) * 0.75, float(vals[-1])]
    return np.array(out, np.float64)


@pytest.mark.parametrize("dtype", [oracle.BF16, oracle.F16])
def test_round_to_half_formats_is_nearest_even(dtype):
    rng = np.random.default_rng(11 + dtype)
    pats, vals = _format_table(dtype)
    lo, hi = (-135, 128) if dtype == oracle.BF16 else (-26, 16)
    v = _probe_values(rng, lo, hi, pats, vals)
    got = oracle.round_values(dtype, v)
    want = np.array([brute_round(float(t), pats, vals) for t in v], np.uint16)
    assert np.array_equal(got, want)


def test_round_f16_and_f32_match_numpy():
    rng = np.random.default_rng(3)
    v = rng.standard_normal(20000) * np.exp2(rng.integers(-30, 20, 20000).astype(np.float64))
    assert np.array_equal(oracle.round_values(oracle.F16, v), v.astype(np.float16).view(np.uint16))
    w = rng.standard_normal(20000) * np.exp2(rng.integers(-160, 130, 20000).astype(np.float64))
    assert np.array_equal(oracle.round_values(oracle.F32, w), w.astype(np.float32).view(np.uint32))


@pytest.mark.parametrize("dtype", [oracle.F32, oracle.BF16, oracle.F16])
def test_widen_is_exact_inverse(dtype):
    rng = np.random.default_rng(4)
    v = rng.standard_normal(5000)
    bits = oracle.round_values(dtype, v)
    w = oracle.widen_values(dtype, bits)
    assert np.array_equal(oracle.round_values(dtype, w), bits)
    if dtype == oracle.F32:
        assert np.array_equal(w, bits.view(np.float32).astype(np.float64))
    elif dtype == oracle.F16:
        assert np.array_equal(w, bits.view(np.float16).astype(np.float64))
    else:
        assert np.array_equal(w, (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64))


# ------------------------------------------------- integer-exact stencils

def test_laplace_64_row_sums():
    """With x = 1 each row sums to 4 - (l_i - 1): 0 inside, 1 on an edge,
    2 at a corner (from the grid position, not from the matrix)."""
    m = gen.laplace_64x64()
    y = oracle.spmv_crs(m.n, m.irp, m.icol, m.val, np.ones(m.n))
    i = np.arange(m.n)
    bx = (i % 64 == 0) | (i % 64 == 63)
    by = (i // 64 == 0) | (i // 64 == 63)
    assert np.array_equal(y, bx.astype(float) + by.astype(float))


def test_stencil27_integer_row_sums():
    e = 20
    m = gen.stencil27(e, e, e, 1, integer_values=True)
    y = oracle.spmv_crs(m.n, m.irp, m.icol, m.val, np.ones(m.n))
    i = np.arange(m.n)
    span = lambda c: np.where((c == 0) | (c == e - 1), 2, 3)
    lens = span(i % e) * span((i // e) % e) * span(i // (e * e))
    assert np.array_equal(y, 27.0 - lens)


def test_validate_flags():
    irp = np.array([0, 2, 3], np.int32)
    icol = np.array([0, 1, 1], np.int32)
    assert oracle.validate_crs(2, irp, icol) == 0
    assert oracle.validate_crs(2, np.array([1, 2, 3], np.int32), icol) & 1
    assert oracle.validate_crs(2, np.array([0, 2, 2], np.int32), icol) & 2
    assert oracle.validate_crs(2, np.array([0, 3, 2], np.int32), icol[:2]) & 4
    assert oracle.validate_crs(2, irp, np.array([0, 2, 1], np.int32)) & 8
    assert oracle.validate_crs(2, irp, np.array([0, -1, 1], np.int32)) & 8
