"""CPU oracle for the run-time CRS transformation and auto-tuning method of
Katagiri & Sato (arXiv:2407.00019).

TEST INFRASTRUCTURE.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library
never links, loads or calls it, and shares no code with it.

The array work lives in ``oracle.c`` (plain single-threaded C, binary64, no
FMA contraction); the scalar formulas of the auto-tuner (Eqs. (1)-(3), the
off-line threshold D* and the on-line decision of section 2.2) are written
below in Python.  Every function cites the passage it follows.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

F64, F32, BF16, F16 = 0, 1, 2, 3
VBYTES = {F64: 8, F32: 4, BF16: 2, F16: 2}


def build() -> None:
    """Compile liboracle.so in place (always recompiles)."""
    subprocess.run(["make", "-B", "-s", "-C", _HERE], check=True)


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64, u64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        lib.orc_validate_crs.argtypes = [i32, i64, P, P]
        lib.orc_validate_crs.restype = ctypes.c_int
        lib.orc_row_moments.argtypes = [i32, P, P, P, P, P]
        lib.orc_bandwidth.argtypes = [i32, P, P]
        lib.orc_bandwidth.restype = i32
        lib.orc_u128_to_double.argtypes = [u64, u64]
        lib.orc_u128_to_double.restype = f64
        lib.orc_dmat.argtypes = [i32, i64, i64, P, P, P]
        lib.orc_expand_ptr.argtypes = [i32, P, P]
        lib.orc_csr_to_ccs.argtypes = [i32, P, P, P, ctypes.c_int, P, P, P]
        lib.orc_csr_to_ccs.restype = ctypes.c_int
        lib.orc_max_len.argtypes = [i32, P]
        lib.orc_max_len.restype = i32
        lib.orc_to_ell.argtypes = [i32, P, P, P, ctypes.c_int, i32, P, P]
        lib.orc_spmv_crs.argtypes = [i32, P, P, P, P, P]
        lib.orc_spmv_coo_row.argtypes = [i32, i64, P, P, P, P, P]
        lib.orc_spmv_ell_row.argtypes = [i32, i32, P, P, P, P]
        lib.orc_spmv_coo_col.argtypes = [i32, i64, P, P, P, P, P]
        lib.orc_spmv_ell_col.argtypes = [i32, i32, P, P, P, P]
        lib.orc_round_values.argtypes = [ctypes.c_int, i64, P, P]
        lib.orc_widen_values.argtypes = [ctypes.c_int, i64, P, P]
        _LIB = lib
    return _LIB


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _raw(val):
    """Values as a contiguous array plus their element size in bytes."""
    a = np.ascontiguousarray(val)
    return a, a.dtype.itemsize


# ------------------------------------------------------------------- input

def validate_crs(n, irp, icol) -> int:
    """CRS contract of section 2.1 (0-based): 0 when valid, else a bit mask
    (1 irp[0] != 0, 2 irp[n] != nnz, 4 irp decreasing, 8 column out of
    range)."""
    irp, icol = _i32(irp), _i32(icol)
    return _lib().orc_validate_crs(n, icol.shape[0], _p(irp), _p(icol))


# ------------------------------------------------------------ Eq. (4) D_mat

def row_moments(n, irp):
    """(s1, s2, max, min) of the row lengths l_i = irp[i+1] - irp[i]."""
    irp = _i32(irp)
    s1, s2 = ctypes.c_int64(), ctypes.c_int64()
    hi, lo = ctypes.c_int32(), ctypes.c_int32()
    _lib().orc_row_moments(n, _p(irp), ctypes.byref(s1), ctypes.byref(s2), ctypes.byref(hi), ctypes.byref(lo))
    return s1.value, s2.value, hi.value, lo.value


def bandwidth(n, irp, icol) -> int:
    """Matrix bandwidth: the largest |i - j| over every stored entry (a
    locality feature of the cost model, not part of the paper)."""
    return int(_lib().orc_bandwidth(n, _p(_i32(irp)), _p(_i32(icol))))


def u128_to_double(v: int) -> float:
    return _lib().orc_u128_to_double(v >> 64, v & ((1 << 64) - 1))


def dmat_from_moments(n, s1, s2):
    """Eq. (4): (mu, sigma, D_mat) with D_mat = sigma / mu over row lengths."""
    mu, sg, d = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _lib().orc_dmat(n, s1, s2, ctypes.byref(mu), ctypes.byref(sg), ctypes.byref(d))
    return mu.value, sg.value, d.value


def dmat(n, irp):
    s1, s2, _, _ = row_moments(n, irp)
    return dmat_from_moments(n, s1, s2)[2]


# --------------------------------------------------- section 2.1 transforms

def csr_to_coo_row(n, irp):
    """COO-Row: IROW, one row index per stored entry (VAL and ICOL are the
    CRS arrays themselves)."""
    irp = _i32(irp)
    out = np.empty(int(irp[n]), np.int32)
    _lib().orc_expand_ptr(n, _p(irp), _p(out))
    return out


def csr_to_ccs(n, irp, icol, val):
    """Phase I, CRS -> CCS: (ccp[n+1], irow_t[nnz], val_t[nnz]), entries of
    a column by row, then by storage position within the row."""
    irp, icol = _i32(irp), _i32(icol)
    v, vb = _raw(val)
    nnz = icol.shape[0]
    ccp = np.empty(n + 1, np.int32)
    irow_t = np.empty(nnz, np.int32)
    val_t = np.empty(nnz, v.dtype)
    if _lib().orc_csr_to_ccs(n, _p(irp), _p(icol), _p(v), vb, _p(ccp), _p(irow_t), _p(val_t)) != 0:
        raise MemoryError("oracle CCS: out of host memory")
    return ccp, irow_t, val_t


def ccs_to_coo_col(n, ccp):
    """Phase II, CCS -> COO-Column: the column index of every entry."""
    return csr_to_coo_row(n, ccp)


def max_len(n, ptr):
    return int(_lib().orc_max_len(n, _p(_i32(ptr))))


def to_ell(n, ptr, idx, val, width=None):
    """ELL of a compressed-line matrix: (ell_val[width*n], ell_idx[width*n]),
    slot-major (slot k of line i at k*n + i), padding value +0.0 and index
    i.  CRS input gives ELL-Row; CCS input gives ELL-Column."""
    ptr, idx = _i32(ptr), _i32(idx)
    v, vb = _raw(val)
    if width is None:
        width = max_len(n, ptr)
    ev = np.empty(width * n, v.dtype)
    ei = np.empty(width * n, np.int32)
    _lib().orc_to_ell(n, _p(ptr), _p(idx), _p(v), vb, width, _p(ev), _p(ei))
    return ev, ei


def csr_to_ell_row(n, irp, icol, val):
    return to_ell(n, irp, icol, val)


def ccs_to_ell_col(n, ccp, irow_t, val_t):
    return to_ell(n, ccp, irow_t, val_t)


# ------------------------------------------------------------------ SpMV

def spmv_crs(n, irp, icol, val, x):
    y = np.empty(n, np.float64)
    _lib().orc_spmv_crs(n, _p(_i32(irp)), _p(_i32(icol)), _p(_f64(val)), _p(_f64(x)), _p(y))
    return y


def spmv_coo_row(n, irow, icol, val, x):
    y = np.empty(n, np.float64)
    irow = _i32(irow)
    _lib().orc_spmv_coo_row(n, irow.shape[0], _p(irow), _p(_i32(icol)), _p(_f64(val)), _p(_f64(x)), _p(y))
    return y


def spmv_ell_row(n, width, ell_val, ell_col, x):
    y = np.empty(n, np.float64)
    _lib().orc_spmv_ell_row(n, width, _p(_f64(ell_val)), _p(_i32(ell_col)), _p(_f64(x)), _p(y))
    return y


def spmv_coo_col(n, jcol, irow_t, val_t, x):
    y = np.empty(n, np.float64)
    jcol = _i32(jcol)
    _lib().orc_spmv_coo_col(n, jcol.shape[0], _p(jcol), _p(_i32(irow_t)), _p(_f64(val_t)), _p(_f64(x)), _p(y))
    return y


def spmv_ell_col(n, width, ell_val, ell_row, x):
    y = np.empty(n, np.float64)
    _lib().orc_spmv_ell_col(n, width, _p(_f64(ell_val)), _p(_i32(ell_row)), _p(_f64(x)), _p(y))
    return y


# ------------------------------------------- reduced-precision value storage

_STORE = {F32: np.uint32, BF16: np.uint16, F16: np.uint16}


def round_values(dtype, v):
    """Round binary64 values to binary32 / bfloat16 / binary16 bit patterns,
    to nearest, ties to even, straight from binary64."""
    v = _f64(v)
    out = np.empty(v.shape[0], _STORE[dtype])
    _lib().orc_round_values(dtype, v.shape[0], _p(v), _p(out))
    return out


def widen_values(dtype, bits):
    bits = np.ascontiguousarray(bits, dtype=_STORE[dtype])
    out = np.empty(bits.shape[0], np.float64)
    _lib().orc_widen_values(dtype, bits.shape[0], _p(bits), _p(out))
    return out


# ------------------------------------------------- section 2.2 auto-tuning

def speedup(t_crs: float, t_fmt: float) -> float:
    """Eq. (1): SP = t_crs / t_ell."""
    return t_crs / t_fmt


def transform_cost(t_trans: float, t_crs: float) -> float:
    """Eq. (2), read as the transformation time in units of one CRS SpMV:
    TT = t_trans / t_crs.  (The printed ratio is the reciprocal; the worked
    example under Eq. (3) and the Fig. 7 definition fix this reading.)"""
    return t_trans / t_crs


def r_ell(sp: float, tt: float) -> float:
    """Eq. (3): R = SP / TT."""
    return sp / tt


def d_star(points, c: float = 1.0) -> float:
    """Off-line phase step (4) of section 2.2: the threshold D* from the
    D_mat-R_ell graph.  `points` are (D_mat, R_ell, feasible) triples.
    Reading: walking the points by increasing D_mat, D* is the first D_mat
    whose R_ell falls below c; +inf when none does.  Infeasible points (the
    format did not fit in memory, like torso1 in section 4.2) are left out.
    Equal D_mat values with mixed outcomes count as a failure at that D_mat."""
    fails = [d for (d, r, ok) in points if ok and not (r >= c)]
    return min(fails) if fails else math.inf


def choose_paper(d_mat: float, dstar: float) -> str:
    """On-line phase of section 2.2: ELL when D_mat < D*, otherwise CRS."""
    return "ell_row" if d_mat < dstar else "crs"


def choose_k_aware(k: int, t_crs: float, candidates: dict, margin: float = 1.0) -> str:
    """Amortised decision over k SpMVs (the iteration-count discussion of
    section 2.2): `candidates` maps a name to (t_trans, t_spmv); the one
    minimising t_trans + k t_spmv (the first in name order on a tie) is
    taken if margin times its cost is below k * t_crs, the cost of staying
    in CRS; otherwise 'crs'."""
    best, cost = None, float("inf")
    for name in sorted(candidates):
        tt, ts = candidates[name]
        c = tt + k * ts
        if c < cost:
            best, cost = name, c
    return best if best is not None and margin * cost < k * t_crs else "crs"


def rel_l2(y, yref) -> float:
    """Relative L2 error ||y - yref|| / ||yref||."""
    y = np.asarray(y, np.float64)
    yref = np.asarray(yref, np.float64)
    den = float(np.linalg.norm(yref))
    num = float(np.linalg.norm(y - yref))
    return num / den if den > 0 else num
