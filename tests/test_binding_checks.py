"""The Python binding refuses, before any library call, tensors that would
make a kernel read or write out of bounds or through a host address: arrays
on the CPU, non-contiguous views, the wrong element type, arrays shorter than
the call needs.  Runs without a GPU: every case raises before the library
touches the device."""
import pytest
import torch

import paper_2407_00019_amd as spmvat


def _cpu(n, dtype):
    return torch.zeros(n, dtype=dtype)


def test_plan_create_refuses_host_tensors():
    n, nnz = 8, 10
    irp, icol = _cpu(n + 1, torch.int32), _cpu(nnz, torch.int32)
    val, ws = _cpu(nnz, torch.float64), _cpu(64, torch.uint8)
    with pytest.raises(spmvat.SpmvArgError) as ei:
        spmvat.spmv_plan_create(n, nnz, irp, icol, val, spmvat.F64, ws)
    assert ei.value.status == spmvat.SPMV_E_ARG and "GPU tensor" in str(ei.value)
    with pytest.raises(spmvat.SpmvArgError):
        spmvat.Plan(irp, icol, val)


def test_plan_create_refuses_unknown_value_type():
    with pytest.raises(spmvat.SpmvArgError):
        spmvat.spmv_plan_create(4, 0, None, None, None, 9, None)
    with pytest.raises(spmvat.SpmvArgError):
        spmvat.Plan(_cpu(5, torch.int32), _cpu(0, torch.int32), _cpu(0, torch.int64))


def test_checks_cover_type_length_and_layout():
    # _dev is the one check every entry point applies to a tensor argument;
    # its device test comes first, so the other conditions are exercised on
    # a tensor that reports itself as a GPU tensor
    class FakeCuda(torch.Tensor):
        @property
        def is_cuda(self):
            return True

    def fake(t):
        return t.as_subclass(FakeCuda)

    ok = fake(torch.zeros(10, dtype=torch.float32))
    spmvat._dev(ok, "t", "x", torch.float32, 10)
    with pytest.raises(spmvat.SpmvArgError, match="must be torch.float64"):
        spmvat._dev(ok, "t", "x", torch.float64, 10)
    with pytest.raises(spmvat.SpmvArgError, match="needs at least 11"):
        spmvat._dev(ok, "t", "x", torch.float32, 11)
    strided = fake(torch.zeros(20, dtype=torch.float32)[::2])
    with pytest.raises(spmvat.SpmvArgError, match="contiguous"):
        spmvat._dev(strided, "t", "x", torch.float32, 10)
    with pytest.raises(spmvat.SpmvArgError, match="torch tensor"):
        spmvat._dev([1.0, 2.0], "t", "x")
    # raw integer addresses are the C ABI's contract and pass through
    spmvat._dev(0x1000, "t", "x", torch.float64, 10)


def test_transformations_refuse_host_buffers():
    out = [_cpu(10, torch.int32)]
    for call in (lambda: spmvat.csr_to_coo(None, 0, out), lambda: spmvat.csr_to_ell(None, 0, out * 2),
                 lambda: spmvat.csr_to_ccs(None, out * 3, _cpu(16, torch.uint8))):
        with pytest.raises(spmvat.SpmvArgError):
            call()


def test_convert_values_refuses_host_and_short_outputs():
    with pytest.raises(spmvat.SpmvArgError):
        spmvat.spmv_convert_values(_cpu(4, torch.float64), _cpu(4, torch.float32), spmvat.F32)
    with pytest.raises(spmvat.SpmvArgError):
        spmvat.spmv_convert_values(_cpu(4, torch.float64), _cpu(4, torch.float32), spmvat.F64)


def test_vector_type_follows_value_storage():
    assert spmvat.vector_dtype(spmvat.F64) == torch.float64
    for t in (spmvat.F32, spmvat.BF16, spmvat.F16):
        assert spmvat.vector_dtype(t) == torch.float32


def test_overlap():
    a = torch.zeros(10)
    assert spmvat._overlap(a[:6], a[5:])
    assert not spmvat._overlap(a[:5], a[5:])
