"""Reduced-precision value storage on the GPU (binary32, bfloat16, binary16
values; binary32 x, y and accumulation), against the CPU oracle.

Stored and transformed value arrays must be bit-exact with the oracle's
round-to-nearest-even.  SpMV is checked row by row against the oracle's
binary64 product of the *stored* values and the binary32 x, with the
forward error bound of a length-l dot product in binary32:
|y_i - y*_i| <= gamma_(l_i + 1) sum_j |a_ij x_j|,  gamma_k = k u / (1 - k u),
u = 2^-24, for every format and order of accumulation."""
import numpy as np
import pytest

import gen
import oracle
from _gpu import higham_ok, host, lib_ready, oracle_transforms, stored_bits

pytestmark = pytest.mark.gpu

MATS = [
    ("laplace64", lambda: gen.laplace_64x64()),
    ("stencil27_e20", lambda: gen.stencil27(20, 20, 20, 3)),
    ("rand_unsorted_dups", lambda: gen.random_small(4000, 9, 12, False, True, 0.2, integer_values=False)),
    ("powerlaw_small", lambda: gen.lognormal_matrix(60000, 16.0, 1.2, 11, 1, 3000)),
    # odd n and n = 2 mod 4, next to the multiples of 4 above
    ("rand_n3001", lambda: gen.random_small(3001, 12, 40, True, False, 0.1, integer_values=False)),
    ("rand_n4002", lambda: gen.random_small(4002, 13, 40, False, False, 0.1, integer_values=False)),
    # the D_mat-sweep shape at full size (n = 1,048,576, 32 per row, D_mat = 0)
    ("dsweep_local_d0", lambda: gen.dsweep_matrix(0, local=True)),
    # bandwidth ~ n = 100,000: the column kernels' row windows exceed the LDS page table
    ("wide_sparse", lambda: gen.random_small(100000, 7, 3, True, False, 0.1, integer_values=False)),
]
DTYPES = [(1, "f32"), (2, "bf16"), (3, "f16")]


@pytest.mark.parametrize("dt,dname", DTYPES, ids=[d[1] for d in DTYPES])
@pytest.mark.parametrize("name,builder", MATS, ids=[m[0] for m in MATS])
def test_reduced_precision_path(name, builder, dt, dname):
    import torch
    spmvat = lib_ready()
    m = builder()
    n = m.n
    dev = torch.device("cuda:0")
    x64 = gen.x_uniform(n, 5)
    x32_bits = oracle.round_values(oracle.F32, x64)
    xw = oracle.widen_values(oracle.F32, x32_bits)
    bits_ref = oracle.round_values(dt, m.val)
    vw = oracle.widen_values(dt, bits_ref)

    irp = torch.from_numpy(m.irp).to(dev)
    icol = torch.from_numpy(m.icol).to(dev)
    val = spmvat.convert_values(torch.from_numpy(m.val).to(dev), dt)
    assert np.array_equal(stored_bits(val), bits_ref)
    xd = torch.from_numpy(xw.astype(np.float32)).to(dev)

    plan = spmvat.Plan(irp, icol, val)
    plan.set_limit(1 << 40)
    (irow,) = plan.to_coo()
    ccp, irow_t, val_t = plan.to_ccs()
    (jcol,) = plan.to_coo(column_wise=True)
    (ev, ec), w = plan.to_ell()
    (cv, cr), wc = plan.to_ell(column_wise=True)
    # transformed values are moved as raw elements: compare bit patterns
    o = oracle_transforms(m, bits_ref)
    assert np.array_equal(host(irow), o["irow"])
    assert np.array_equal(host(ccp), o["ccp"])
    assert np.array_equal(host(irow_t), o["irow_t"])
    assert np.array_equal(stored_bits(val_t), o["val_t"])
    assert np.array_equal(host(jcol), o["jcol"])
    assert np.array_equal(stored_bits(ev), o["ell_val"])
    assert np.array_equal(host(ec), o["ell_col"])
    assert np.array_equal(stored_bits(cv), o["ellc_val"])
    assert np.array_equal(host(cr), o["ellc_row"])

    yref = oracle.spmv_crs(n, m.irp, m.icol, vw, xw)
    absref = oracle.spmv_crs(n, m.irp, m.icol, np.abs(vw), np.abs(xw))
    lens = np.diff(m.irp)
    for fmt, var in [(spmvat.CRS, 0), (spmvat.CRS, 1), (spmvat.CRS, 5), (spmvat.CRS, 8), (spmvat.COO_ROW, 0),
                     (spmvat.ELL_ROW, 0), (spmvat.COO_COL, 0), (spmvat.COO_COL, 1), (spmvat.COO_COL, 2),
                     (spmvat.ELL_COL, 0), (spmvat.ELL_COL, 1), (spmvat.ELL_COL, 2)]:
        y = plan.spmv(fmt, xd, variant=var)
        assert y.dtype == torch.float32
        ok = higham_ok(host(y), yref, absref, lens)
        assert ok.all(), (name, dname, fmt, var, int((~ok).sum()))
    plan.close()
