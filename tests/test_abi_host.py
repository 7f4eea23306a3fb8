"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/spmvat.h declares, and its host-only logic (status strings, the
off-line D* rule, the on-line format choice) agrees with the oracle.  No
device work is done here."""
import math
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_2407_00019_amd as spmvat
    if not os.path.exists(spmvat.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return spmvat


def declared_functions():
    text = open(os.path.join(ROOT, "include", "spmvat.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    spmvat = _lib()
    names = declared_functions()
    assert len(names) >= 16
    L = spmvat.lib()
    for name in names:
        assert hasattr(L, name), name


def test_status_strings():
    spmvat = _lib()
    assert spmvat.status_string(0) == "ok"
    assert "limit" in spmvat.status_string(spmvat.SPMV_E_TOO_LARGE)
    assert spmvat.status_string(99) == "unknown status"


def test_plan_create_rejects_sizes_before_touching_the_gpu():
    """n < 1, nnz < 0, nnz above SPMV_MAX_NNZ (2^31 - 2^20: headroom for the
    kernels' 32-bit position steps) and an unknown value type are refused
    with SPMV_E_ARG before any allocation, so this runs without a GPU."""
    import ctypes
    spmvat = _lib()
    L = spmvat.lib()
    with open(os.path.join(ROOT, "include", "spmvat.h")) as fh:
        assert f"#define SPMV_MAX_NNZ {spmvat.MAX_NNZ}" in fh.read()
    dummy = ctypes.c_void_p(16)   # never dereferenced: the sizes are checked first
    for n, nnz, dt in ((0, 0, 0), (10, -1, 0), (10, spmvat.MAX_NNZ + 1, 0), (10, 2**31 - 1, 1), (10, 5, 7)):
        h = ctypes.c_void_p()
        s = L.spmv_plan_create(ctypes.byref(h), n, nnz, dummy, dummy, dummy, dt, dummy, 1 << 20, None)
        assert s == spmvat.SPMV_E_ARG, (n, nnz, dt)
        assert not h.value


def test_workspace_size_grows_with_nnz():
    spmvat = _lib()
    a = spmvat.spmv_plan_workspace_bytes(10, 100)
    b = spmvat.spmv_plan_workspace_bytes(10, 10_000_000)
    assert a > 0 and b > a and b % 256 == 0


@pytest.mark.parametrize("seed", range(40))
def test_dstar_matches_oracle(seed):
    spmvat = _lib()
    rng = np.random.default_rng(seed)
    m = int(rng.integers(0, 12))
    d = np.round(rng.uniform(0, 4, m), 2).tolist()
    if m > 2:
        d[1] = d[0]          # ties
    r = rng.uniform(0, 3, m).tolist()
    feas = (rng.random(m) > 0.2).astype(int).tolist()
    t = spmvat.at_table_build(d, r, feas, 1.0)
    want = oracle.d_star(list(zip(d, r, [bool(f) for f in feas])), 1.0)
    assert t.d_star == want
    assert t.c == 1.0


def _stats(n, nnz, max_row, d_mat, bandwidth=100):
    spmvat = _lib()
    st = spmvat.spmv_stats()
    st.n, st.nnz, st.max_row, st.min_row, st.max_col = n, nnz, max_row, 1, -1
    st.bandwidth = bandwidth
    st.sum_len = nnz
    st.mu = nnz / n
    st.d_mat = d_mat
    return st


def test_paper_rule_and_memory_guard():
    spmvat = _lib()
    t = spmvat.at_table_build([0.1, 0.5, 1.0], [2.0, 0.8, 0.1], None, 1.0)
    assert t.d_star == 0.5
    st = _stats(1000, 27000, 27, 0.07)
    f, v, why = spmvat.at_choose_format_stats(st, spmvat.F64, 1 << 40, t, 0)
    assert (f, v, why.rule, why.feasible_ell) == (spmvat.ELL_ROW, 0, 0, 1)
    st.d_mat = 0.5
    assert spmvat.at_choose_format_stats(st, spmvat.F64, 1 << 40, t, 0)[0] == spmvat.CRS
    st.d_mat = 0.07
    # ELL-Row needs 27 * 1000 * 12 bytes: refuse below that
    f, v, why = spmvat.at_choose_format_stats(st, spmvat.F64, 27 * 1000 * 12 - 1, t, 0)
    assert f == spmvat.CRS and why.feasible_ell == 0
    assert spmvat.at_choose_format_stats(st, spmvat.F64, 27 * 1000 * 12, t, 0)[0] == spmvat.ELL_ROW


def _calibrated(spmvat, crs0, crs1, coo, ell, tr_coo, tr_ell, launch=0.0, loc=(0, 1), buckets=None):
    t = spmvat.at_table_build([], [], None, 1.0)
    t.calibrated = 1
    for l in loc:
        for b in (range(spmvat.AT_DBUCKETS) if buckets is None else buckets):
            t.spmv_bps[l][spmvat.CRS][0][b] = crs0
            t.spmv_bps[l][spmvat.CRS][1][b] = crs1
            t.spmv_bps[l][spmvat.COO_ROW][0][b] = coo
            t.spmv_bps[l][spmvat.ELL_ROW][0][b] = ell
            t.trans_bps[l][spmvat.COO_ROW][b] = tr_coo
            t.trans_bps[l][spmvat.ELL_ROW][b] = tr_ell
    t.launch_s = launch
    return t


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 20, 100, 500])
@pytest.mark.parametrize("dtype", [0, 1, 2])
def test_k_aware_choice_matches_oracle(k, dtype):
    """The library's amortised choice equals the oracle's argmin of
    t_trans + k t_spmv over the same estimates (bytes / rate + launches)."""
    spmvat = _lib()
    n, nnz, w = 100000, 2_600_000, 27
    st = _stats(n, nnz, w, 0.07)
    vb = {0: 8, 1: 4, 2: 2}[dtype]
    xb = 8 if dtype == 0 else 4
    t = _calibrated(spmvat, 2.0e12, 3.0e12, 2.5e12, 4.0e12, 3.0e12, 2.0e12, 2e-6)
    crs_b = (vb + 4) * nnz + 4 * (n + 1) + 2 * xb * n
    coo_b = (vb + 8) * nnz + 2 * xb * n
    ell_b = (vb + 4) * n * w + 2 * xb * n
    tcrs = min(crs_b / 2.0e12, crs_b / 3.0e12) + 2e-6
    cands = {
        "coo_row": ((4 * (n + 1) + 4 * nnz) / 3.0e12 + 2e-6, coo_b / 2.5e12 + 4e-6),
        "ell_row": (((vb + 4) * nnz + 4 * (n + 1) + ell_b - 2 * xb * n) / 2.0e12 + 2e-6, ell_b / 4.0e12 + 2e-6),
    }
    want = oracle.choose_k_aware(k, tcrs, cands, spmvat.AT_K_MARGIN)
    f, v, why = spmvat.at_choose_format_stats(st, dtype, 1 << 40, t, k)
    got = {spmvat.CRS: "crs", spmvat.COO_ROW: "coo_row", spmvat.ELL_ROW: "ell_row"}[f]
    assert got == want
    assert why.rule == 1
    if got == "crs":
        assert v == 1        # the faster CRS variant
    else:
        ts = cands[got][1]
        assert why.k_break_even == pytest.approx((cands[got][0] / tcrs) / (1 - ts / tcrs))


def test_k_aware_needs_a_gain_beyond_the_margin():
    """A transformation predicted to save less than the margin keeps CRS;
    one predicted to save more converts.  The constant is the header's."""
    spmvat = _lib()
    with open(os.path.join(ROOT, "include", "spmvat.h")) as fh:
        hdr = fh.read()
    assert f"#define AT_K_MARGIN {spmvat.AT_K_MARGIN}" in hdr
    n, nnz, w = 100000, 2_600_000, 26
    st = _stats(n, nnz, w, 0.0)
    crs_b = 12 * nnz + 4 * (n + 1) + 16 * n
    ell_b = 12 * n * w + 16 * n
    for gain, want in ((1.05, spmvat.CRS), (1.2, spmvat.ELL_ROW)):
        # ELL-Row `gain` times faster per byte-normalised SpMV, transformation free
        ell_rate = 1e12 * gain * ell_b / crs_b
        t = _calibrated(spmvat, 1e12, 1e12, 1e9, ell_rate, 1e9, 1e30)
        f, v, why = spmvat.at_choose_format_stats(st, 0, 1 << 40, t, 1000)
        assert f == want, (gain, f)
        cands = {"ell_row": (0.0, crs_b / 1e12 / gain)}
        want_o = "crs" if want == spmvat.CRS else "ell_row"
        assert oracle.choose_k_aware(1000, crs_b / 1e12, cands, spmvat.AT_K_MARGIN) == want_o


def test_table_margin_replaces_the_default():
    """A table that carries its own margin (measured by the off-line phase)
    decides with it: a 15% predicted gain converts under the default 1.1
    and keeps CRS under a measured 1.2, as the oracle's rule says."""
    spmvat = _lib()
    n, nnz, w = 100000, 2_600_000, 26
    st = _stats(n, nnz, w, 0.0)
    crs_b = 12 * nnz + 4 * (n + 1) + 16 * n
    ell_b = 12 * n * w + 16 * n
    ell_rate = 1e12 * 1.15 * ell_b / crs_b
    cands = {"ell_row": (0.0, crs_b / 1e12 / 1.15)}
    for margin, want in ((0.0, spmvat.ELL_ROW), (1.2, spmvat.CRS), (1.1, spmvat.ELL_ROW)):
        t = _calibrated(spmvat, 1e12, 1e12, 1e9, ell_rate, 1e9, 1e30)
        t.k_margin = margin
        f, v, why = spmvat.at_choose_format_stats(st, 0, 1 << 40, t, 1000)
        assert f == want, (margin, f)
        used = margin if margin > 0 else spmvat.AT_K_MARGIN
        want_o = oracle.choose_k_aware(1000, crs_b / 1e12, cands, used)
        assert want_o == ("crs" if want == spmvat.CRS else "ell_row")


def test_off_line_table_is_stamped_with_the_kernel_sources():
    """The committed auto-tuning table names the kernel sources it was
    measured with (a hash of the sources of the kernels the off-line phase
    times), carries a measured margin, and the library's JSON reader takes
    the margin over."""
    import json
    spmvat = _lib()
    with open(os.path.join(ROOT, "paper_2407_00019_amd", "at_table.json")) as f:
        d = json.load(f)
    assert isinstance(d.get("kernel_source_sha"), str) and len(d["kernel_source_sha"]) == 16
    assert spmvat.table_matches_kernels(d) in (True, False)
    # the stamp covers exactly those sources: another file's change leaves it
    assert spmvat.table_kernel_sha() == spmvat.kernel_source_sha(spmvat.TABLE_KERNEL_SOURCES)
    assert spmvat.table_kernel_sha() != spmvat.kernel_source_sha()
    assert d["k_margin"] >= 1.0
    assert spmvat.at_table_from_json(d).k_margin == pytest.approx(d["k_margin"])


def test_committed_measurements_match_the_kernel_sources():
    """The committed auto-tuning table and counter summaries were taken
    with the kernels in this tree: the auto-tuning
    table carries the hash of the off-line phase's kernel sources and the
    HBM traffic table the hash of all kernel sources (bench.py drops its
    traffic figure when they differ)."""
    import json
    spmvat = _lib()
    with open(os.path.join(ROOT, "paper_2407_00019_amd", "at_table.json")) as f:
        assert json.load(f)["kernel_source_sha"] == spmvat.table_kernel_sha()
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        tj = json.load(f)
    assert tj["source_sha"] == spmvat.kernel_source_sha()
    for section in ("kernels", "powerlaw_kernels", "dsweep_kernels", "dsweep_local_kernels"):
        assert tj[section], section
        assert all(e["source_sha"] == tj["source_sha"] for e in tj[section].values())


def test_cost_model_cell_follows_locality_and_d_bucket():
    """The k-aware choice reads the table cell of the matrix's locality class
    (bandwidth <= 65536 or not) and D_mat bucket (edges 1/16, 1/8, 1/4, 1/2,
    1, 2, 4): an ELL rate present in only one cell wins only there."""
    spmvat = _lib()
    edges = spmvat.AT_DBUCKET_EDGES
    for loc in (0, 1):
        for b in range(spmvat.AT_DBUCKETS):
            t = _calibrated(spmvat, 1e12, 1e12, 1e9, 0.0, 1e9, 0.0)
            t.spmv_bps[loc][spmvat.ELL_ROW][0][b] = 1e13
            t.trans_bps[loc][spmvat.ELL_ROW][b] = 1e13
            for l2 in (0, 1):
                for b2 in range(spmvat.AT_DBUCKETS):
                    d = 0.0 if b2 == 0 else edges[b2 - 1]
                    bw = spmvat.AT_LOCAL_BAND if l2 == 0 else spmvat.AT_LOCAL_BAND + 1
                    st = _stats(100000, 2_600_000, 27, d, bandwidth=bw)
                    f, v, why = spmvat.at_choose_format_stats(st, 0, 1 << 40, t, 100)
                    assert (f == spmvat.ELL_ROW) == (l2 == loc and b2 == b), (loc, b, l2, b2)


def test_uncalibrated_table_falls_back_to_paper_rule():
    spmvat = _lib()
    t = spmvat.at_table_build([0.3], [0.5], None, 1.0)
    st = _stats(1000, 5000, 5, 0.2)
    f, v, why = spmvat.at_choose_format_stats(st, 0, 1 << 40, t, 50)
    assert why.rule == 0 and f == spmvat.ELL_ROW
    t2 = spmvat.at_table_build([], [], None, 1.0)
    assert math.isinf(t2.d_star)


def test_arena_first_fit_and_coalescing():
    """The server's offset allocator against a plain Python model of
    first-fit over 256-byte granules with coalescing frees."""
    spmvat = _lib()
    L = spmvat.lib()
    cap = 1 << 20
    A = L.spmv_arena_create(cap)
    model = [(0, cap)]                       # sorted free list (offset, size)

    def m_alloc(b):
        need = max(b, 1)
        need = (need + 255) // 256 * 256
        for i, (o, s) in enumerate(model):
            if s >= need:
                if s == need:
                    model.pop(i)
                else:
                    model[i] = (o + need, s - need)
                return o
        return -1

    def m_free(o, b):
        s = (max(b, 1) + 255) // 256 * 256
        model.append((o, s))
        model.sort()
        merged = []
        for seg in model:
            if merged and merged[-1][0] + merged[-1][1] == seg[0]:
                merged[-1] = (merged[-1][0], merged[-1][1] + seg[1])
            else:
                merged.append(seg)
        model[:] = merged

    rng = np.random.default_rng(0)
    live = []
    for step in range(3000):
        if live and rng.random() < 0.45:
            o, b = live.pop(int(rng.integers(0, len(live))))
            L.spmv_arena_free(A, o, b)
            m_free(o, b)
        else:
            b = int(rng.integers(1, 40000))
            o = L.spmv_arena_alloc(A, b)
            assert o == m_alloc(b)
            if o >= 0:
                live.append((o, b))
        assert L.spmv_arena_free_bytes(A) == sum(s for _, s in model)
        assert L.spmv_arena_largest(A) == max([s for _, s in model] or [0])
    for o, b in live:
        L.spmv_arena_free(A, o, b)
    assert L.spmv_arena_free_bytes(A) == cap and L.spmv_arena_largest(A) == cap
    L.spmv_arena_destroy(A)


def test_noalloc_coo_row_refuses_before_touching_the_gpu():
    """The COO-Row entry point that allocates nothing checks its sizes before
    any HIP call: n < 1 and an unknown type give SPMV_E_ARG, nnz past the
    fixed carry array gives SPMV_E_TOO_LARGE (the header states the limit)."""
    import ctypes
    spmvat = _lib()
    L = spmvat.lib()
    with open(os.path.join(ROOT, "include", "spmvat.h")) as fh:
        assert f"#define SPMV_COO_ROW_NOALLOC_MAX_NNZ {spmvat.COO_ROW_NOALLOC_MAX_NNZ}" in fh.read()
    d = ctypes.c_void_p(256)   # never dereferenced: the sizes are checked first
    f = L.spmv_exec_coo_row_noalloc
    assert f(0, 0, d, d, d, spmvat.F64, d, d, None) == spmvat.SPMV_E_ARG
    assert f(8, -1, d, d, d, spmvat.F64, d, d, None) == spmvat.SPMV_E_ARG
    assert f(8, 8, d, d, d, 7, d, d, None) == spmvat.SPMV_E_ARG
    assert f(8, spmvat.COO_ROW_NOALLOC_MAX_NNZ + 1, d, d, d, spmvat.F32, d, d, None) == spmvat.SPMV_E_TOO_LARGE


def test_arena_refuses_sizes_and_ranges_it_did_not_give():
    """A size whose rounding would wrap, a second free of one block and a
    range outside the arena leave the allocator unchanged."""
    spmvat = _lib()
    L = spmvat.lib()
    cap = 1 << 16
    A = L.spmv_arena_create(cap)
    size_max = 2**64 - 1
    assert L.spmv_arena_alloc(A, size_max) == -1
    assert L.spmv_arena_alloc(A, size_max - 200) == -1
    assert L.spmv_arena_alloc(A, cap + 1) == -1
    o = L.spmv_arena_alloc(A, 1000)
    assert o == 0 and L.spmv_arena_free_bytes(A) == cap - 1024
    L.spmv_arena_free(A, o, 1000)
    L.spmv_arena_free(A, o, 1000)            # already free: ignored
    assert L.spmv_arena_free_bytes(A) == cap and L.spmv_arena_largest(A) == cap
    a = L.spmv_arena_alloc(A, 512)
    b = L.spmv_arena_alloc(A, 512)
    assert (a, b) == (0, 512)
    for off, size in ((-256, 256), (cap, 256), (cap - 256, 512), (0, size_max), (1024, 256)):
        L.spmv_arena_free(A, off, size)      # outside the arena, or free space: ignored
        assert L.spmv_arena_free_bytes(A) == cap - 1024
    L.spmv_arena_free(A, b, 512)
    L.spmv_arena_free(A, a, 512)
    assert L.spmv_arena_free_bytes(A) == cap and L.spmv_arena_largest(A) == cap
    L.spmv_arena_destroy(A)
