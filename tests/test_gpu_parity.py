"""GPU parity: the HIP path, called through the C ABI, against the CPU oracle
on the same seeded inputs.

Bar: index, pointer and transformed value arrays bit-exact; D_mat and its
integer moments bit-exact; binary64 SpMV within relative L2 1e-13 in every
format and variant, and bitwise equal when the data are small integers (all
partial sums exact, so even the atomic formats must agree)."""
import numpy as np
import pytest

import gen
import oracle
from _gpu import F64, bits, host, lib_ready, oracle_transforms, stored_bits, to_dev

pytestmark = pytest.mark.gpu

TOL64 = 1e-13

SMALL = [
    # name, builder
    ("laplace64", lambda: gen.laplace_64x64()),
    ("stencil27_e9", lambda: gen.stencil27(9, 9, 9, 5)),
    ("rand_sorted", lambda: gen.random_small(3001, 1, 12, True, False, 0.1, integer_values=False)),
    ("rand_unsorted", lambda: gen.random_small(2500, 2, 9, False, False, 0.2, integer_values=False)),
    ("rand_dups", lambda: gen.random_small(1700, 3, 9, False, True, 0.3, integer_values=False)),
    ("mostly_empty", lambda: gen.random_small(5000, 4, 3, True, False, 0.9, integer_values=False)),
    ("single_row", lambda: gen.random_small(1, 5, 1, True, False, 0.0, integer_values=False)),
    ("no_entries", lambda: gen.random_small(300, 6, 0, True, False, 0.0, integer_values=False)),
    ("powerlaw_small", lambda: gen.lognormal_matrix(40000, 16.0, 1.2, 7, 1, 4000)),
    ("banded", lambda: gen.banded(7777, 40, 8)),
]


def arrow(n, seed, dense_cols=(0,), mid_col=None, mid_len=1000):
    """Every row holds the dense columns; one more column holds mid_len
    entries; plus a short random part.  Exercises the workgroup and
    multi-pass column sorts."""
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(n):
        c = set(dense_cols)
        if mid_col is not None and i % max(1, n // mid_len) == 0:
            c.add(mid_col)
        c.update(rng.integers(0, n, size=int(rng.integers(0, 4))).tolist())
        rows.append(sorted(c))
    lens = np.array([len(r) for r in rows])
    irp = np.zeros(n + 1, np.int64)
    irp[1:] = np.cumsum(lens)
    icol = np.concatenate([np.array(r, np.int32) for r in rows])
    val = rng.standard_normal(icol.shape[0])
    return gen.Crs(n, irp.astype(np.int32), icol, val, f"arrow_{n}")


SMALL += [
    ("arrow_mid", lambda: arrow(3000, 9, dense_cols=(5,), mid_col=77, mid_len=700)),
    ("arrow_long", lambda: arrow(50000, 10, dense_cols=(0, 49999), mid_col=123, mid_len=5000)),
    # bandwidth ~ n = 100,000: every column workgroup's row window is wider
    # than the page table, so the paged column kernels fall back per workgroup
    ("wide_sparse", lambda: gen.random_small(100000, 7, 3, True, False, 0.1, integer_values=False)),
]


def run_gpu_all(m, x64):
    import torch
    spmvat = lib_ready()
    irp, icol, val = to_dev(m)
    xd = torch.from_numpy(x64).to("cuda:0")
    plan = spmvat.Plan(irp, icol, val)
    plan.set_limit(1 << 40)          # the memory guard has its own test
    out = {"stats": plan.stats}
    (out["irow"],) = plan.to_coo()
    out["ccp"], out["irow_t"], out["val_t"] = plan.to_ccs()
    (out["jcol"],) = plan.to_coo(column_wise=True)
    (out["ell_val"], out["ell_col"]), out["ell_w"] = plan.to_ell()
    (out["ellc_val"], out["ellc_row"]), out["ellc_w"] = plan.to_ell(column_wise=True)
    out["max_col"] = plan.stats.max_col
    ys = {}
    for fmt, var in [(spmvat.CRS, 0), (spmvat.CRS, 1), (spmvat.CRS, 2), (spmvat.CRS, 4), (spmvat.CRS, 6),
                     (spmvat.CRS, 7), (spmvat.CRS, 8), (spmvat.COO_ROW, 0), (spmvat.ELL_ROW, 0),
                     (spmvat.COO_COL, 0), (spmvat.COO_COL, 1), (spmvat.COO_COL, 2),
                     (spmvat.ELL_COL, 0), (spmvat.ELL_COL, 1), (spmvat.ELL_COL, 2)]:
        ys[(fmt, var)] = host(plan.spmv(fmt, xd, variant=var))
    out["y"] = ys
    out = {k: (host(v) if hasattr(v, "cpu") else v) for k, v in out.items()}
    plan.close()
    return out


def check_transforms(m, g, o):
    assert np.array_equal(g["irow"], o["irow"])
    assert np.array_equal(g["ccp"], o["ccp"])
    assert np.array_equal(g["irow_t"], o["irow_t"])
    assert np.array_equal(bits(g["val_t"]), bits(o["val_t"]))
    assert np.array_equal(g["jcol"], o["jcol"])
    assert g["ell_w"] == o["ell_w"]
    assert np.array_equal(bits(g["ell_val"]), bits(o["ell_val"]))
    assert np.array_equal(g["ell_col"], o["ell_col"])
    assert g["ellc_w"] == o["ellc_w"] == g["max_col"]
    assert np.array_equal(bits(g["ellc_val"]), bits(o["ellc_val"]))
    assert np.array_equal(g["ellc_row"], o["ellc_row"])


def check_stats(m, st):
    s1, s2, mx, mn = oracle.row_moments(m.n, m.irp)
    mu, sg, d = oracle.dmat_from_moments(m.n, s1, s2)
    assert (st.sum_len, st.sum_len2, st.max_row, st.min_row) == (s1, s2, mx, mn)
    assert st.bandwidth == oracle.bandwidth(m.n, m.irp, m.icol)
    assert bits(np.array([st.mu, st.sigma, st.d_mat])).tolist() == bits(np.array([mu, sg, d])).tolist()


@pytest.mark.parametrize("name,builder", SMALL, ids=[s[0] for s in SMALL])
def test_small_matrices_full_path(name, builder):
    m = builder()
    x = gen.x_uniform(m.n, 99)
    g = run_gpu_all(m, x)
    check_stats(m, g["stats"])
    check_transforms(m, g, oracle_transforms(m))
    yref = oracle.spmv_crs(m.n, m.irp, m.icol, m.val, x)
    for key, y in g["y"].items():
        assert oracle.rel_l2(y, yref) <= TOL64, (name, key, oracle.rel_l2(y, yref))


INTEGER_CASES = SMALL[:6] + [s for s in SMALL if s[0] in ("powerlaw_small", "banded")]


@pytest.mark.parametrize("name,builder", INTEGER_CASES, ids=[s[0] for s in INTEGER_CASES])
def test_integer_data_is_bitwise_exact(name, builder):
    m = builder()
    rng = np.random.default_rng(3)
    m.val = rng.integers(-5, 6, size=m.nnz).astype(np.float64)
    x = rng.integers(-3, 4, size=m.n).astype(np.float64)
    g = run_gpu_all(m, x)
    yref = oracle.spmv_crs(m.n, m.irp, m.icol, m.val, x)
    for key, y in g["y"].items():
        assert np.array_equal(y, yref), (name, key)


def test_laplace_x_one_exact():
    m = gen.laplace_64x64()
    g = run_gpu_all(m, np.ones(m.n))
    i = np.arange(m.n)
    want = ((i % 64 == 0) | (i % 64 == 63)).astype(float) + ((i // 64 == 0) | (i // 64 == 63)).astype(float)
    for key, y in g["y"].items():
        assert np.array_equal(y, want), key


def test_transforms_and_coo_row_are_deterministic():
    import torch
    spmvat = lib_ready()
    m = gen.lognormal_matrix(200000, 16.0, 1.2, 21, 1, 3000)
    irp, icol, val = to_dev(m)
    x = torch.from_numpy(gen.x_uniform(m.n, 4)).to("cuda:0")
    res = []
    for _ in range(2):
        plan = spmvat.Plan(irp, icol, val)
        ccp, irow_t, val_t = plan.to_ccs()
        (jcol,) = plan.to_coo(column_wise=True)
        plan.to_coo()
        y = plan.spmv(spmvat.COO_ROW, x)
        res.append([host(ccp), host(irow_t), bits(host(val_t)), host(jcol), bits(host(y))])
        plan.close()
    for a, b in zip(*res):
        assert np.array_equal(a, b)


@pytest.mark.slow
def test_stencil27_128_full_size():
    """The headline workload at full size (n = 2,097,152, nnz = 55,742,968),
    the same calls the benchmark times: every array bit-exact, every SpMV
    within 1e-13."""
    m = gen.stencil27_128()
    assert m.nnz == 382 ** 3
    x = gen.x_uniform(m.n, gen.seed_for(2))
    g = run_gpu_all(m, x)
    check_stats(m, g["stats"])
    assert g["ell_w"] == 27 and g["max_col"] == 27
    check_transforms(m, g, oracle_transforms(m))
    yref = oracle.spmv_crs(m.n, m.irp, m.icol, m.val, x)
    for key, y in g["y"].items():
        assert oracle.rel_l2(y, yref) <= TOL64, (key, oracle.rel_l2(y, yref))


@pytest.mark.slow
def test_powerlaw_full_size():
    """n = 4,194,304 lognormal rows (D_mat ~ 1.80): ELL-Row is refused by the
    memory guard; everything else is checked against the oracle."""
    import torch
    spmvat = lib_ready()
    m = gen.powerlaw()
    x = gen.x_uniform(m.n, gen.seed_for(3))
    irp, icol, val = to_dev(m)
    xd = torch.from_numpy(x).to("cuda:0")
    plan = spmvat.Plan(irp, icol, val)
    check_stats(m, plan.stats)
    s, sz = plan.sizes(spmvat.ELL_ROW)
    assert s == spmvat.SPMV_E_TOO_LARGE
    assert sz.width == oracle.max_len(m.n, m.irp)
    with pytest.raises(spmvat.SpmvError) as ei:
        plan.to_ell()
    assert ei.value.status == spmvat.SPMV_E_TOO_LARGE
    (irow,) = plan.to_coo()
    ccp, irow_t, val_t = plan.to_ccs()
    (jcol,) = plan.to_coo(column_wise=True)
    (cv, cr), wc = plan.to_ell(column_wise=True)
    o_irow = oracle.csr_to_coo_row(m.n, m.irp)
    o_ccp, o_irow_t, o_val_t = oracle.csr_to_ccs(m.n, m.irp, m.icol, m.val)
    assert np.array_equal(host(irow), o_irow)
    assert np.array_equal(host(ccp), o_ccp)
    assert np.array_equal(host(irow_t), o_irow_t)
    assert np.array_equal(bits(host(val_t)), bits(o_val_t))
    assert np.array_equal(host(jcol), oracle.ccs_to_coo_col(m.n, o_ccp))
    o_cv, o_cr = oracle.to_ell(m.n, o_ccp, o_irow_t, o_val_t)
    assert wc == oracle.max_len(m.n, o_ccp)
    assert np.array_equal(bits(host(cv)), bits(o_cv))
    assert np.array_equal(host(cr), o_cr)
    yref = oracle.spmv_crs(m.n, m.irp, m.icol, m.val, x)
    for fmt, var in [(spmvat.CRS, 0), (spmvat.CRS, 1), (spmvat.CRS, 5), (spmvat.CRS, 8), (spmvat.COO_ROW, 0),
                     (spmvat.COO_COL, 0), (spmvat.COO_COL, 2), (spmvat.ELL_COL, 0), (spmvat.ELL_COL, 2)]:
        y = host(plan.spmv(fmt, xd, variant=var))
        assert oracle.rel_l2(y, yref) <= TOL64, (fmt, var)
    plan.close()


@pytest.mark.slow
@pytest.mark.parametrize("local", [False, True], ids=["scattered", "local"])
def test_dsweep_d0_full_size(local):
    """The D_mat-sweep shape at full size (n = 1,048,576, 32 entries per row,
    D_mat = 0) in both column families, through every transformation and
    SpMV the off-line phase times: arrays bit-exact, SpMV within 1e-13."""
    m = gen.dsweep_matrix(0, local=local)
    x = gen.x_uniform(m.n, gen.seed_for(5, 100))
    g = run_gpu_all(m, x)
    check_stats(m, g["stats"])
    assert g["ell_w"] == 32
    check_transforms(m, g, oracle_transforms(m))
    yref = oracle.spmv_crs(m.n, m.irp, m.icol, m.val, x)
    for key, y in g["y"].items():
        assert oracle.rel_l2(y, yref) <= TOL64, (key, oracle.rel_l2(y, yref))


@pytest.mark.slow
def test_dsweep_d1_full_size_without_ell_row():
    """A high-D_mat sweep matrix at full size (scattered columns, D_mat = 1):
    ELL-Row is refused by the default memory guard; the statistics, COO-Row,
    CCS, COO-Column and ELL-Column arrays are bit-exact and every SpMV that
    can run is within 1e-13."""
    import torch
    spmvat = lib_ready()
    m = gen.dsweep_matrix(8)
    x = gen.x_uniform(m.n, gen.seed_for(5, 108))
    irp, icol, val = to_dev(m)
    xd = torch.from_numpy(x).to("cuda:0")
    plan = spmvat.Plan(irp, icol, val)
    check_stats(m, plan.stats)
    assert abs(plan.stats.d_mat - 1.0) < 1e-4
    s, _ = plan.sizes(spmvat.ELL_ROW)
    assert s == spmvat.SPMV_E_TOO_LARGE
    (irow,) = plan.to_coo()
    ccp, irow_t, val_t = plan.to_ccs()
    (jcol,) = plan.to_coo(column_wise=True)
    (cv, cr), wc = plan.to_ell(column_wise=True)
    # the oracle's arrays one by one (its ELL-Row would be ~1700 slots wide)
    o_ccp, o_irow_t, o_val_t = oracle.csr_to_ccs(m.n, m.irp, m.icol, m.val)
    assert np.array_equal(host(irow), oracle.csr_to_coo_row(m.n, m.irp))
    assert np.array_equal(host(ccp), o_ccp)
    assert np.array_equal(host(irow_t), o_irow_t)
    assert np.array_equal(bits(host(val_t)), bits(o_val_t))
    assert np.array_equal(host(jcol), oracle.ccs_to_coo_col(m.n, o_ccp))
    o_cv, o_cr = oracle.to_ell(m.n, o_ccp, o_irow_t, o_val_t)
    assert wc == oracle.max_len(m.n, o_ccp)
    assert np.array_equal(bits(host(cv)), bits(o_cv)) and np.array_equal(host(cr), o_cr)
    yref = oracle.spmv_crs(m.n, m.irp, m.icol, m.val, x)
    for fmt, var in [(spmvat.CRS, 0), (spmvat.CRS, 1), (spmvat.CRS, 6), (spmvat.COO_ROW, 0),
                     (spmvat.COO_COL, 0), (spmvat.ELL_COL, 0)]:
        y = host(plan.spmv(fmt, xd, variant=var))
        assert oracle.rel_l2(y, yref) <= TOL64, (fmt, var)
    plan.close()


def banded_with_long_column(n, seed):
    """Band of half-width 2 plus column 0 in every 8th row from row 8 on:
    column 0 then holds those rows and rows 0-2 of the band."""
    m = gen.banded(n, 2, seed)
    rows = np.arange(8, n, 8)
    at = m.irp[rows]
    icol = np.insert(m.icol, at, 0)
    val = np.insert(m.val, at, np.random.default_rng(seed).standard_normal(rows.shape[0]))
    extra = np.zeros(n + 1, np.int64)
    extra[rows + 1] = 1
    irp = (m.irp + np.cumsum(extra)).astype(np.int32)
    return gen.Crs(n, irp, icol.astype(np.int32), val, f"banded_long_n{n}")


@pytest.mark.slow
@pytest.mark.parametrize("n", [1 << 22, (1 << 22) + 3001])
def test_ccs_with_a_long_column_at_large_n(n):
    """n around 2^22 with one column of n / 8 entries (the multi-pass column
    sort): the oracle's arrays bit for bit."""
    import torch
    spmvat = lib_ready()
    m = banded_with_long_column(n, 31)
    assert oracle.validate_crs(m.n, m.irp, m.icol) == 0
    x = gen.x_uniform(m.n, 5)
    irp, icol, val = to_dev(m)
    plan = spmvat.Plan(irp, icol, val)
    ccp, irow_t, val_t = plan.to_ccs()
    (jcol,) = plan.to_coo(column_wise=True)
    o_ccp, o_irow_t, o_val_t = oracle.csr_to_ccs(m.n, m.irp, m.icol, m.val)
    assert plan.stats.max_col == int(np.diff(o_ccp).max()) == len(range(8, n, 8)) + 3
    assert np.array_equal(host(ccp), o_ccp)
    assert np.array_equal(host(irow_t), o_irow_t)
    assert np.array_equal(bits(host(val_t)), bits(o_val_t))
    assert np.array_equal(host(jcol), oracle.ccs_to_coo_col(m.n, o_ccp))
    yref = oracle.spmv_crs(m.n, m.irp, m.icol, m.val, x)
    y = host(plan.spmv(spmvat.COO_COL, torch.from_numpy(x).to("cuda:0")))
    assert oracle.rel_l2(y, yref) <= TOL64
    plan.close()


@pytest.mark.slow
@pytest.mark.parametrize("n", [64 * 131072, 64 * 131072 + 3001])
def test_ccs_banded_at_the_block_scan_limit(n):
    """The banded CRS -> CCS at n = 8,388,608 (131,072 column blocks: the most
    one workgroup scans, in eight chunks) and 3,001 rows past it (the shared
    multi-kernel scan takes the block counts): the oracle's arrays bit for
    bit."""
    spmvat = lib_ready()
    m = gen.banded(n, 2, 41)
    irp, icol, val = to_dev(m)
    plan = spmvat.Plan(irp, icol, val)
    ccp, irow_t, val_t = plan.to_ccs(algorithm=spmvat.CCS_BANDED)
    o_ccp, o_irow_t, o_val_t = oracle.csr_to_ccs(m.n, m.irp, m.icol, m.val)
    assert np.array_equal(host(ccp), o_ccp)
    assert np.array_equal(host(irow_t), o_irow_t)
    assert np.array_equal(bits(host(val_t)), bits(o_val_t))
    assert plan.stats.max_col == int(np.diff(o_ccp).max())
    plan.close()


def test_error_paths_leave_the_plan_usable():
    import torch
    spmvat = lib_ready()
    m = gen.laplace_64x64()
    irp, icol, val = to_dev(m)
    dev = irp.device
    ws = torch.empty(spmvat.spmv_plan_workspace_bytes(m.n, m.nnz), dtype=torch.uint8, device=dev)
    # malformed CRS
    bad_col = icol.clone()
    bad_col[17] = m.n
    for args in [(irp, bad_col, val), (irp + 1, icol, val)]:
        with pytest.raises(spmvat.SpmvError) as ei:
            spmvat.spmv_plan_create(m.n, m.nnz, *args, spmvat.F64, ws)
        assert ei.value.status == spmvat.SPMV_E_MATRIX
    dec = irp.clone()
    dec[10], dec[11] = dec[11].item(), dec[10].item()
    with pytest.raises(spmvat.SpmvError) as ei:
        spmvat.spmv_plan_create(m.n, m.nnz, dec, icol, val, spmvat.F64, ws)
    assert ei.value.status == spmvat.SPMV_E_MATRIX
    # misaligned pointer
    with pytest.raises(spmvat.SpmvError) as ei:
        spmvat.spmv_plan_create(m.n, m.nnz - 1, irp, icol[1:], val[1:], spmvat.F64, ws)
    assert ei.value.status == spmvat.SPMV_E_ARG
    plan = spmvat.Plan(irp, icol, val)
    x = torch.from_numpy(gen.x_uniform(m.n, 1)).to(dev)
    for fmt in (spmvat.COO_ROW, spmvat.ELL_ROW, spmvat.COO_COL, spmvat.ELL_COL):
        with pytest.raises(spmvat.SpmvError) as ei:
            plan.spmv(fmt, x)
        assert ei.value.status == spmvat.SPMV_E_NOT_READY
    with pytest.raises(spmvat.SpmvError) as ei:
        plan.to_coo(column_wise=True)
    assert ei.value.status == spmvat.SPMV_E_NOT_READY
    plan.to_ell()
    plan.set_limit(1000)
    with pytest.raises(spmvat.SpmvError) as ei:
        plan.to_ccs()
    assert ei.value.status == spmvat.SPMV_E_TOO_LARGE
    # the ELL-Row built before the refusal still works
    yref = oracle.spmv_crs(m.n, m.irp, m.icol, m.val, host(x))
    assert oracle.rel_l2(host(plan.spmv(spmvat.ELL_ROW, x)), yref) <= TOL64
    # short output buffer
    plan.set_limit(1 << 40)
    s, sz = plan.sizes(spmvat.COO_ROW)
    short = torch.empty(sz.bytes[0] // 4 - 1, dtype=torch.int32, device=dev)
    with pytest.raises(spmvat.SpmvError) as ei:
        spmvat.csr_to_coo(plan.handle, 0, [short])
    assert ei.value.status == spmvat.SPMV_E_ARG
    plan.close()


def test_convert_values_bits_match_oracle():
    import torch
    spmvat = lib_ready()
    rng = np.random.default_rng(12)
    v = np.concatenate([
        rng.standard_normal(100000),
        rng.standard_normal(20000) * np.exp2(rng.integers(-160, 130, 20000).astype(np.float64)),
        np.array([0.0, -0.0, 65504.0, 65519.99, 65520.0, 1e6, -1e6, 5.96e-8, 2.98e-8, 1e-300, 3.4e38, 3.5e38]),
    ])
    # exact ties between neighbouring bfloat16 / binary16 values and one step either side
    for step_exp in (-7, -10):
        base = 1.0 + np.arange(1, 200) * 2.0 ** step_exp
        mid = base + 2.0 ** (step_exp - 1)
        v = np.concatenate([v, mid, np.nextafter(mid, 2), np.nextafter(mid, 0)])
    vd = torch.from_numpy(v).to("cuda:0")
    for dt in (spmvat.F32, spmvat.BF16, spmvat.F16):
        got = stored_bits(spmvat.convert_values(vd, dt))
        want = oracle.round_values(dt, v)
        assert np.array_equal(got, want), dt
        # short arrays and ragged tails: four values a thread, the rest one by one
        for m in list(range(1, 10)) + [v.shape[0] - 3]:
            got = stored_bits(spmvat.convert_values(vd[:m].contiguous(), dt))
            assert np.array_equal(got, want[:m]), (dt, m)


def band_edges(n, bw, seed):
    """Rows i with columns i-1, i, i+1 and i - bw, i + bw where they exist,
    plus a dense row: bandwidth exactly bw, sorted rows."""
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    cols = [i - bw, i - 1, i, i + 1, i + bw]
    mask = [(c >= 0) & (c < n) for c in cols]
    lens = np.sum(mask, axis=0)
    dense = n // 2
    extra = np.arange(max(0, dense - bw), min(n, dense + bw + 1), 97)
    rows = []
    for r in range(n):
        c = [int(cc[r]) for cc, mm in zip(cols, mask) if mm[r]]
        if r == dense:
            c = sorted(set(c) | set(extra.tolist()))
        rows.append(c)
    lens = np.array([len(r) for r in rows])
    irp = np.zeros(n + 1, np.int64)
    irp[1:] = np.cumsum(lens)
    icol = np.concatenate([np.array(r, np.int32) for r in rows])
    return gen.Crs(n, irp.astype(np.int32), icol, rng.standard_normal(icol.shape[0]), f"band_edges_{bw}")


@pytest.mark.parametrize("bw", [17888, 17900, 17921])
def test_ccs_around_the_privatised_window_limits(bw):
    """Column counts are privatised in LDS up to bandwidth 17920, the scatter
    up to 17888: matrices on both sides of each limit give the oracle's CCS
    bit for bit, and the bandwidth statistic is exact."""
    spmvat = lib_ready()
    m = band_edges(60000, bw, 40 + bw)
    assert oracle.bandwidth(m.n, m.irp, m.icol) == bw
    irp, icol, val = to_dev(m)
    plan = spmvat.Plan(irp, icol, val)
    assert plan.stats.bandwidth == bw
    ccp, irow_t, val_t = plan.to_ccs()
    o_ccp, o_irow_t, o_val_t = oracle.csr_to_ccs(m.n, m.irp, m.icol, m.val)
    assert np.array_equal(host(ccp), o_ccp)
    assert np.array_equal(host(irow_t), o_irow_t)
    assert np.array_equal(bits(host(val_t)), bits(o_val_t))
    assert plan.stats.max_col == int(np.diff(o_ccp).max())
    plan.close()


def _stream_lanes(n, nnz):
    # the stream kernel's lanes per row, restated from its launch rule: one
    # per 32 entries of the mean row, doubled while the grid holds fewer than
    # 1024 workgroups of 256/G rows and a lane keeps at least four entries
    mean = nnz / n
    g = 1
    while g < 64 and 64 * g <= mean:
        g *= 2
    while g < 64 and n * g // 256 < 1024 and 8 * g <= mean:
        g *= 2
    return g


@pytest.mark.parametrize("lanes,mean", [(1, 5), (2, 10), (4, 20), (8, 40), (16, 80), (32, 160), (64, 300)])
def test_stream_crs_every_lane_count(lanes, mean):
    """The stream CRS kernel at each lanes-per-row count it can pick, on rows
    around the mean plus empty rows and rows longer than 256 entries (summed
    by the whole workgroup) at workgroup edges: binary64 within 1e-13 of the
    oracle, bitwise on small-integer data."""
    import torch
    spmvat = lib_ready()
    n = 3000
    rng = np.random.default_rng(lanes)
    lengths = np.clip(rng.poisson(mean, n), 0, n).astype(np.int32)
    rows = 256 // lanes
    for r in (0, 1, rows - 1, rows, n // 2, n - 1):
        lengths[r] = 700 if r % 2 == 0 else 300
    lengths[[5, rows + 1, n - 2]] = 0
    m = gen.random_rows(n, lengths, 40 + lanes)
    assert _stream_lanes(n, int(m.irp[-1])) == lanes
    for integer in (False, True):
        val = np.round(m.val * 4) if integer else m.val
        mm = gen.Crs(n, m.irp, m.icol, val, m.name)
        x64 = np.round(gen.x_uniform(n, 9) * 8) if integer else gen.x_uniform(n, 9)
        irp, icol, vd = to_dev(mm)
        xd = torch.from_numpy(x64).to("cuda:0")
        plan = spmvat.Plan(irp, icol, vd)
        yref = oracle.spmv_crs(n, mm.irp, mm.icol, mm.val, x64)
        for variant in (1, 8):
            y = host(plan.spmv(spmvat.CRS, xd, variant=variant))
            if integer:
                assert np.array_equal(y, yref), (lanes, variant)
            else:
                assert oracle.rel_l2(y, yref) <= TOL64, (lanes, variant)
        plan.close()


def _ell_parts(n, width):
    # threads per row of ELL-Row, restated from its launch rule: doubled
    # while the grid holds fewer than 1024 workgroups and each thread keeps
    # at least four slots, at most 16
    p = 1
    while p < 16 and n * p // 256 < 1024 and 8 * p <= width:
        p *= 2
    return p


@pytest.mark.parametrize("parts,width", [(1, 5), (2, 12), (4, 20), (8, 40), (16, 100)])
def test_ell_row_outer_parallel_every_split(parts, width):
    """ELL-Row with a row's slots split over 1..16 threads (Fig. 4's
    outer-parallel form) on rows of every length up to the width, empty rows
    included: binary64 within 1e-13 of the oracle's Fig. 3 loop, bitwise on
    small-integer data; the ELL arrays themselves stay bit-exact."""
    import torch
    spmvat = lib_ready()
    n = 3000
    rng = np.random.default_rng(100 + parts)
    lengths = rng.integers(0, width + 1, n).astype(np.int32)
    lengths[[0, n // 2, n - 1]] = width
    lengths[[1, 7]] = 0
    m = gen.random_rows(n, lengths, 60 + parts)
    assert _ell_parts(n, int(lengths.max())) == parts
    for integer in (False, True):
        val = np.round(m.val * 4) if integer else m.val
        mm = gen.Crs(n, m.irp, m.icol, val, m.name)
        x64 = np.round(gen.x_uniform(n, 11) * 8) if integer else gen.x_uniform(n, 11)
        irp, icol, vd = to_dev(mm)
        xd = torch.from_numpy(x64).to("cuda:0")
        plan = spmvat.Plan(irp, icol, vd)
        (ev, ec), w = plan.to_ell()
        want_v, want_c = oracle.csr_to_ell_row(n, mm.irp, mm.icol, mm.val)[:2]
        assert w == width
        assert np.array_equal(bits(host(ev)), bits(want_v)) and np.array_equal(host(ec), want_c)
        y = host(plan.spmv(spmvat.ELL_ROW, xd))
        yref = oracle.spmv_ell_row(n, w, want_v, want_c, x64)
        if integer:
            assert np.array_equal(y, yref), parts
        else:
            assert oracle.rel_l2(y, yref) <= TOL64, parts
        plan.close()


def _integer_copy(m, seed):
    """The same sparsity pattern with small-integer values, so every partial
    sum of an SpMV is exact."""
    v = np.random.default_rng(seed).integers(-4, 5, m.nnz).astype(np.float64)
    return gen.Crs(m.n, m.irp, m.icol, v, m.name + "_int")


@pytest.mark.slow
@pytest.mark.parametrize("local", [False, True], ids=["scattered", "local"])
def test_dsweep_wide_ell_row_full_size(local):
    """The D_mat-sweep point D = 0.125 at full size (n = 1,048,576): binary64
    ELL-Row rows wider than the unrolled kernels cover (Fig. 3 with the slot
    loop taken at run time, two rows per thread), the kernel the off-line
    phase times there.  ELL arrays bit-exact with the oracle; SpMV within
    1e-13 of the oracle's Fig. 3 loop, and bitwise on small-integer data."""
    import torch
    spmvat = lib_ready()
    m = gen.dsweep_matrix(1, local=local)
    w_o = oracle.max_len(m.n, m.irp)
    # the launch rule takes one thread per row (n fills the GPU), two rows
    # per thread (n even) and the run-time slot loop (width > 32)
    assert m.n % 2 == 0 and w_o > 32 and _ell_parts(m.n, w_o) == 1
    x = gen.x_uniform(m.n, gen.seed_for(5, 201))
    xi = np.round(x * 3)
    for mm, xx, exact in ((m, x, False), (_integer_copy(m, 77), xi, True)):
        irp, icol, val = to_dev(mm)
        xd = torch.from_numpy(xx).to("cuda:0")
        plan = spmvat.Plan(irp, icol, val)
        check_stats(mm, plan.stats)
        (ev, ec), w = plan.to_ell()
        assert w == w_o
        o_ev, o_ec = oracle.csr_to_ell_row(mm.n, mm.irp, mm.icol, mm.val)
        assert np.array_equal(bits(host(ev)), bits(o_ev))
        assert np.array_equal(host(ec), o_ec)
        y = host(plan.spmv(spmvat.ELL_ROW, xd))
        yref = oracle.spmv_ell_row(mm.n, w, o_ev, o_ec, xx)
        if exact:
            assert np.array_equal(y, yref)
        else:
            assert oracle.rel_l2(y, yref) <= TOL64
        del o_ev, o_ec
        plan.close()


def dup_long_column(n, reps, seed):
    """Every row holds column 7 `reps` times (duplicates, kept as separate
    entries) plus 0-3 random columns, rows unsorted: column 7 then holds
    reps * n entries, more than n and than a workgroup's sort."""
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(n):
        c = [7] * reps + rng.integers(0, n, size=int(rng.integers(0, 4))).tolist()
        rng.shuffle(c)
        rows.append(c)
    lens = np.array([len(r) for r in rows])
    irp = np.zeros(n + 1, np.int64)
    irp[1:] = np.cumsum(lens)
    icol = np.concatenate([np.array(r, np.int32) for r in rows])
    return gen.Crs(n, irp.astype(np.int32), icol, rng.standard_normal(icol.shape[0]), f"dup_long_{n}x{reps}")


@pytest.mark.parametrize("n,reps", [(3000, 3), (9000, 2)])
def test_ccs_duplicate_column_longer_than_n(n, reps):
    """A column with more entries than the matrix has rows (only possible
    with duplicates) and than one workgroup sorts: CCS, COO-Column and
    ELL-Column bit-exact with the oracle, the duplicates in row, then
    storage order; SpMV within 1e-13."""
    import torch
    spmvat = lib_ready()
    m = dup_long_column(n, reps, 300 + n)
    assert oracle.validate_crs(m.n, m.irp, m.icol) == 0
    x = gen.x_uniform(n, 12)
    g = run_gpu_all(m, x)
    o = oracle_transforms(m)
    assert g["max_col"] >= reps * n > max(n, 8192)
    check_transforms(m, g, o)
    yref = oracle.spmv_crs(m.n, m.irp, m.icol, m.val, x)
    for key, y in g["y"].items():
        assert oracle.rel_l2(y, yref) <= TOL64, (key, oracle.rel_l2(y, yref))


def wide_random_rows(n, per_row, seed):
    """Sorted random rows of `per_row` columns each over all n columns: a
    512-row tile then touches more columns than the windowed placement keeps
    in LDS."""
    rng = np.random.default_rng(seed)
    icol = np.empty(n * per_row, np.int32)
    for i in range(n):
        icol[i * per_row:(i + 1) * per_row] = np.sort(rng.choice(n, per_row, replace=False))
    irp = np.arange(0, n * per_row + 1, per_row, dtype=np.int32)
    return gen.Crs(n, irp, icol, rng.standard_normal(icol.shape[0]), f"wide_random_{n}x{per_row}")


CCS_CASES = {
    "stencil27_e12": lambda: gen.stencil27(12, 12, 12, 3),
    "band_edges_3000": lambda: band_edges(20000, 3000, 76),
    "dup_long": lambda: dup_long_column(600, 128, 77),
    "wide_random": lambda: wide_random_rows(60000, 150, 78),
    "rand_unsorted": lambda: gen.random_small(2500, 2, 9, False, False, 0.2, integer_values=False),
}


@pytest.mark.parametrize("alg", ["sort", "bucketed", "banded", "radix"])
@pytest.mark.parametrize("case", sorted(CCS_CASES))
def test_ccs_every_algorithm(case, alg):
    """Each CRS -> CCS algorithm, selected on the plan, on matrices of every
    kind: a stencil, a band at its edges, a column of 76,800 duplicate
    entries (longer than n: the sort ranks it across sorted chunks), random
    rows over 60,000 columns, unsorted rows.  CCS and COO-Column bit-exact
    with the oracle, the longest column right, COO-Column SpMV within 1e-13."""
    import torch
    spmvat = lib_ready()
    m = CCS_CASES[case]()
    assert oracle.validate_crs(m.n, m.irp, m.icol) == 0
    irp, icol, val = to_dev(m)
    plan = spmvat.Plan(irp, icol, val)
    code = {"sort": spmvat.CCS_SORT, "bucketed": spmvat.CCS_BUCKETED, "banded": spmvat.CCS_BANDED,
            "radix": spmvat.CCS_RADIX}[alg]
    ccp, irow_t, val_t = plan.to_ccs(algorithm=code)
    (jcol,) = plan.to_coo(column_wise=True)
    o_ccp, o_irow_t, o_val_t = oracle.csr_to_ccs(m.n, m.irp, m.icol, m.val)
    assert np.array_equal(host(ccp), o_ccp)
    assert np.array_equal(host(irow_t), o_irow_t)
    assert np.array_equal(bits(host(val_t)), bits(o_val_t))
    assert np.array_equal(host(jcol), oracle.ccs_to_coo_col(m.n, o_ccp))
    assert plan.stats.max_col == int(np.diff(o_ccp).max())
    x = gen.x_uniform(m.n, 13)
    yref = oracle.spmv_crs(m.n, m.irp, m.icol, m.val, x)
    y = host(plan.spmv(spmvat.COO_COL, torch.from_numpy(x).to("cuda:0")))
    assert oracle.rel_l2(y, yref) <= TOL64
    plan.close()


def test_banded_ccs_reports_an_entry_outside_the_measured_band():
    """The banded CRS -> CCS relies on the bandwidth measured when the plan
    was made: after one column index moves far outside that band it reports
    SPMV_E_MATRIX instead of a wrong CCS, and once the index is back the
    same plan converts bit-exactly."""
    spmvat = lib_ready()
    m = gen.banded(20000, 3, 43)
    irp, icol, val = to_dev(m)
    plan = spmvat.Plan(irp, icol, val)
    assert plan.stats.bandwidth == 3
    p = int(m.irp[100]) + 1
    kept = int(icol[p].item())
    icol[p] = 15000
    with pytest.raises(spmvat.SpmvError) as ei:
        plan.to_ccs(algorithm=spmvat.CCS_BANDED)
    assert ei.value.status == spmvat.SPMV_E_MATRIX
    icol[p] = kept
    ccp, irow_t, val_t = plan.to_ccs(algorithm=spmvat.CCS_BANDED)
    o_ccp, o_irow_t, o_val_t = oracle.csr_to_ccs(m.n, m.irp, m.icol, m.val)
    assert np.array_equal(host(ccp), o_ccp)
    assert np.array_equal(host(irow_t), o_irow_t)
    assert np.array_equal(bits(host(val_t)), bits(o_val_t))
    plan.close()


def one_per_row(n, seed):
    """One entry per row at a random column: nnz = n exactly."""
    rng = np.random.default_rng(seed)
    irp = np.arange(n + 1, dtype=np.int32)
    icol = rng.integers(0, n, size=n).astype(np.int32)
    return gen.Crs(n, irp, icol, rng.standard_normal(n), f"one_per_row_{n}")


RADIX_CASES = {
    # one, two and three 8-bit passes, and the edges of tiles of 2048 entries
    "n200_one_pass": lambda: gen.random_small(200, 31, 9, False, True, 0.1, integer_values=False),
    "n257_two_passes": lambda: gen.random_small(257, 32, 30, True, False, 0.2, integer_values=False),
    "n70000_three_passes": lambda: gen.random_small(70000, 33, 12, False, False, 0.1, integer_values=False),
    "nnz_2048": lambda: one_per_row(2048, 34),
    "nnz_2049": lambda: one_per_row(2049, 35),
    "nnz_4097": lambda: one_per_row(4097, 36),
    "no_entries": lambda: gen.random_small(300, 6, 0, True, False, 0.0, integer_values=False),
    "single_row": lambda: gen.random_small(1, 5, 1, True, False, 0.0, integer_values=False),
}


@pytest.mark.parametrize("case", sorted(RADIX_CASES))
def test_ccs_radix_passes(case):
    """The radix CRS -> CCS with one, two and three digit passes, tiles cut
    at and across 2048 entries, no entries, one row: CCS bit-exact with the
    oracle and the longest column right."""
    spmvat = lib_ready()
    m = RADIX_CASES[case]()
    assert oracle.validate_crs(m.n, m.irp, m.icol) == 0
    irp, icol, val = to_dev(m)
    plan = spmvat.Plan(irp, icol, val)
    ccp, irow_t, val_t = plan.to_ccs(algorithm=spmvat.CCS_RADIX)
    o_ccp, o_irow_t, o_val_t = oracle.csr_to_ccs(m.n, m.irp, m.icol, m.val)
    assert np.array_equal(host(ccp), o_ccp)
    assert np.array_equal(host(irow_t), o_irow_t)
    assert np.array_equal(bits(host(val_t)), bits(o_val_t))
    assert plan.stats.max_col == (int(np.diff(o_ccp).max()) if m.n else 0)
    plan.close()


@pytest.mark.parametrize("case", sorted(RADIX_CASES))
def test_ccs_banded_small_and_ragged(case):
    """The banded CRS -> CCS on the small cases of the radix test: tiles
    holding fewer entries than waves (empty stretches, stretches shorter
    than one 16-byte quad), one row, one entry per row; no entries takes
    the plain route.  CCS bit-exact with the oracle."""
    spmvat = lib_ready()
    m = RADIX_CASES[case]()
    irp, icol, val = to_dev(m)
    plan = spmvat.Plan(irp, icol, val)
    ccp, irow_t, val_t = plan.to_ccs(algorithm=spmvat.CCS_BANDED)
    o_ccp, o_irow_t, o_val_t = oracle.csr_to_ccs(m.n, m.irp, m.icol, m.val)
    assert np.array_equal(host(ccp), o_ccp)
    assert np.array_equal(host(irow_t), o_irow_t)
    assert np.array_equal(bits(host(val_t)), bits(o_val_t))
    assert plan.stats.max_col == (int(np.diff(o_ccp).max()) if m.n else 0)
    plan.close()


@pytest.mark.parametrize("case", ["stencil27_e12", "dup_long", "rand_unsorted"])
def test_ccs_in_place_copy_back(case):
    """The in-place CCS (Phase I with its copy-back): the plan's own CRS
    tensors end up holding the oracle's column pointers, row numbers and
    values bit for bit; COO-Column and ELL-Column built from them match the
    oracle, COO-Column SpMV is within 1e-13, and CRS SpMV is refused."""
    import torch
    spmvat = lib_ready()
    m = CCS_CASES[case]()
    irp, icol, val = to_dev(m)
    plan = spmvat.Plan(irp, icol, val)
    plan.set_limit(1 << 40)
    ccp, irow_t, val_t = plan.to_ccs_inplace()
    assert ccp.data_ptr() == irp.data_ptr() and irow_t.data_ptr() == icol.data_ptr()
    o_ccp, o_irow_t, o_val_t = oracle.csr_to_ccs(m.n, m.irp, m.icol, m.val)
    assert np.array_equal(host(irp), o_ccp)
    assert np.array_equal(host(icol), o_irow_t)
    assert np.array_equal(bits(host(val)), bits(o_val_t))
    (jcol,) = plan.to_coo(column_wise=True)
    assert np.array_equal(host(jcol), oracle.ccs_to_coo_col(m.n, o_ccp))
    (cv, cr), wc = plan.to_ell(column_wise=True)
    o_cv, o_cr = oracle.ccs_to_ell_col(m.n, o_ccp, o_irow_t, o_val_t)
    assert np.array_equal(bits(host(cv)), bits(o_cv)) and np.array_equal(host(cr), o_cr)
    x = gen.x_uniform(m.n, 14)
    xd = torch.from_numpy(x).to("cuda:0")
    yref = oracle.spmv_crs(m.n, m.irp, m.icol, m.val, x)
    assert oracle.rel_l2(host(plan.spmv(spmvat.COO_COL, xd)), yref) <= TOL64
    with pytest.raises(spmvat.SpmvError) as e:
        plan.spmv(spmvat.CRS, xd, variant=8)
    assert e.value.status == spmvat.SPMV_E_NOT_READY
    torch.cuda.synchronize()
    plan.close()


def test_binding_refuses_vectors_that_do_not_fit_the_plan():
    """x and y of the wrong element type, too short, on the host, strided or
    overlapping are refused by the binding before any kernel runs, and the
    plan stays usable."""
    import torch
    spmvat = lib_ready()
    m = gen.laplace_64x64()
    irp, icol, val = to_dev(m)
    plan = spmvat.Plan(irp, icol, val)
    dev = irp.device
    x = torch.from_numpy(gen.x_uniform(m.n, 3)).to(dev)
    bad = [
        (x.float(), torch.empty_like(x)),                           # binary32 x on a binary64 plan
        (x, torch.empty(m.n - 1, dtype=torch.float64, device=dev)),  # short y
        (x.cpu(), torch.empty_like(x)),                             # host x
        (torch.empty(2 * m.n, dtype=torch.float64, device=dev)[::2], torch.empty_like(x)),  # strided
        (x, x),                                                     # x and y overlap
    ]
    for xx, yy in bad:
        with pytest.raises(spmvat.SpmvArgError):
            spmvat.spmv_exec(plan.handle, spmvat.CRS, 1, xx, yy)
    yref = oracle.spmv_crs(m.n, m.irp, m.icol, m.val, host(x))
    assert oracle.rel_l2(host(plan.spmv(spmvat.CRS, x, variant=1)), yref) <= TOL64
    # a plan over reduced-precision values takes binary32 vectors
    p32 = spmvat.Plan(irp, icol, spmvat.convert_values(val, spmvat.F32))
    with pytest.raises(spmvat.SpmvArgError):
        p32.spmv(spmvat.CRS, x)
    y32 = host(p32.spmv(spmvat.CRS, x.float(), variant=1))
    assert np.all(np.isfinite(y32))
    p32.close()
    plan.close()
