"""Shared helpers of the GPU parity tests: run the HIP path and the oracle on
the same seeded inputs and compare."""
import numpy as np

import oracle

F64, F32, BF16, F16 = 0, 1, 2, 3


def lib_ready():
    import os
    import paper_2407_00019_amd as spmvat
    if not os.path.exists(spmvat.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return spmvat


def to_dev(m, dtype=F64):
    """Device copies of a host CRS; values converted on the GPU when reduced."""
    import torch
    spmvat = lib_ready()
    dev = torch.device("cuda:0")
    irp = torch.from_numpy(np.ascontiguousarray(m.irp)).to(dev)
    icol = torch.from_numpy(np.ascontiguousarray(m.icol)).to(dev)
    val64 = torch.from_numpy(np.ascontiguousarray(m.val)).to(dev)
    if dtype == F64:
        return irp, icol, val64
    return irp, icol, spmvat.convert_values(val64, dtype)


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def bits(a):
    a = np.asarray(a)
    return a.view({8: np.uint64, 4: np.uint32, 2: np.uint16}[a.dtype.itemsize])


def stored_bits(t):
    """Bit pattern of a device value tensor (any float type)."""
    import torch
    torch.cuda.synchronize()
    if t.dtype in (torch.bfloat16, torch.float16):
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return bits(t.cpu().numpy())


def oracle_transforms(m, val=None):
    """Every transformed array the oracle produces for matrix m (values
    `val`, default m.val, moved as raw elements)."""
    v = m.val if val is None else val
    n = m.n
    out = {"irow": oracle.csr_to_coo_row(n, m.irp)}
    ccp, irow_t, val_t = oracle.csr_to_ccs(n, m.irp, m.icol, v)
    out.update(ccp=ccp, irow_t=irow_t, val_t=val_t, jcol=oracle.ccs_to_coo_col(n, ccp))
    out["ell_w"] = oracle.max_len(n, m.irp)
    out["ell_val"], out["ell_col"] = oracle.to_ell(n, m.irp, m.icol, v)
    out["ellc_w"] = oracle.max_len(n, ccp)
    out["ellc_val"], out["ellc_row"] = oracle.to_ell(n, ccp, irow_t, val_t)
    return out


def higham_ok(y, yref, absref, lens, u=2.0 ** -24):
    """Per-row forward error bound of a length-l dot product in a format
    with unit roundoff u: |y - yref| <= gamma_(l+1) sum |a x|, with
    gamma_k = k u / (1 - k u) (plus 1e-15 of slack for the binary64
    reference itself)."""
    k = lens.astype(np.float64) + 1.0
    gamma = k * u / (1.0 - k * u)
    err = np.abs(np.asarray(y, np.float64) - yref)
    bound = gamma * absref + 1e-15 * absref + 1e-300
    return err <= bound
