"""The COO-Row SpMV entry point that allocates nothing
(spmv_exec_coo_row_noalloc), through the C ABI, against spmv_exec(COO_ROW)
on a plan: bitwise equal on two calls in a row, the second with a smaller
matrix (the fixed carry array keeps the first call's contents), in every
value type; sizes past the array's limit are refused before any work."""
import numpy as np
import pytest

import gen
import oracle
from _gpu import F64, F32, BF16, F16, bits, host, lib_ready, to_dev

pytestmark = pytest.mark.gpu


def _case(m, dtype, seed):
    import torch
    spmvat = lib_ready()
    irp, icol, val = to_dev(m, dtype)
    vt = spmvat.vector_dtype(dtype)
    x = torch.from_numpy(gen.x_uniform(m.n, seed)).to("cuda:0").to(vt)
    plan = spmvat.Plan(irp, icol, val)
    (irow,) = plan.to_coo()
    y_plan = plan.spmv(spmvat.COO_ROW, x)
    # a y full of garbage: the entry point must clear the rows without entries
    y_static = torch.full((m.n,), float("nan"), dtype=vt, device="cuda:0")
    spmvat.spmv_exec_coo_row_noalloc(m.n, icol.numel(), irow, icol, val, dtype, x, y_static)
    yp, ys = host(y_plan), host(y_static)
    plan.close()
    return m, x, yp, ys


@pytest.mark.parametrize("dtype", [F64, F32, BF16, F16])
def test_noalloc_matches_plan_path_twice(dtype):
    big = gen.lognormal_matrix(60000, 24.0, 1.0, 31, 0, 9000)    # empty rows, rows spanning workgroups
    small = gen.random_small(3001, 32, 12, True, False, 0.2, integer_values=False)
    for m, seed in ((big, 1), (small, 2)):
        print(f"noalloc case {m.name} n={m.n} nnz={m.icol.size} dtype={dtype}", flush=True)
        m, x, yp, ys = _case(m, dtype, seed)
        assert np.array_equal(bits(yp), bits(ys)), m.name
        if dtype == F64:
            ref = oracle.spmv_crs(m.n, m.irp, m.icol, m.val, host(x))
            assert oracle.rel_l2(ys, ref) <= 1e-13


def test_noalloc_refuses_sizes_past_its_array():
    import torch
    spmvat = lib_ready()
    dummy = torch.zeros(16, dtype=torch.float64, device="cuda:0")
    L = spmvat.lib()
    p = dummy.data_ptr()
    too_many = spmvat.COO_ROW_NOALLOC_MAX_NNZ + 1
    assert L.spmv_exec_coo_row_noalloc(4, too_many, p, p, p, F64, p, p, None) == spmvat.SPMV_E_TOO_LARGE
    assert L.spmv_exec_coo_row_noalloc(0, 0, p, p, p, F64, p, p, None) == spmvat.SPMV_E_ARG
    assert L.spmv_exec_coo_row_noalloc(4, 4, p + 8, p, p, F64, p, p, None) == spmvat.SPMV_E_ARG
