"""Python binding of libspmvat (include/spmvat.h): run-time CRS -> COO / CCS /
ELL transformation, SpMV in every format, and the D_mat / R_ell auto-tuner of
Katagiri & Sato (arXiv:2407.00019), on AMD MI355X.

The functions below carry the C ABI's names and only marshal arguments:
torch tensors become device pointers, torch's current stream becomes the
hipStream_t.  Every step runs in the HIP library; if it is not built, loading
raises (there is no fallback).  ``Plan`` is a convenience owner that
allocates the caller-owned device buffers as torch tensors and keeps them
alive as long as the plan.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import torch  # first: its HIP runtime is the one the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libspmvat.so")
_LIB = None

# enums of spmvat.h
SPMV_OK, SPMV_E_ARG, SPMV_E_MATRIX, SPMV_E_TOO_LARGE, SPMV_E_NOT_READY, SPMV_E_HIP = range(6)
CRS, COO_ROW, CCS, COO_COL, ELL_ROW, ELL_COL = range(6)
CCS_AUTO, CCS_SORT, CCS_BUCKETED, CCS_BANDED, CCS_RADIX = range(5)   # spmv_ccs_algorithm
F64, F32, BF16, F16 = range(4)
FORMAT_NAMES = {CRS: "crs", COO_ROW: "coo_row", CCS: "ccs", COO_COL: "coo_col", ELL_ROW: "ell_row",
                ELL_COL: "ell_col"}
DTYPE_OF_TORCH = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16, torch.float16: F16}
TORCH_OF_DTYPE = {v: k for k, v in DTYPE_OF_TORCH.items()}
AT_DBUCKETS = 8
AT_LOCAL_BAND = 65536
AT_K_MARGIN = 1.1        # the k-aware rule's required predicted gain (spmvat.h)
MAX_NNZ = 2**31 - 2**20  # SPMV_MAX_NNZ: headroom for the kernels' 32-bit position steps
AT_DBUCKET_EDGES = (0.0625, 0.125, 0.25, 0.5, 1.0, 2.0, 4.0)


class SpmvError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str = ""):
        self.status = status
        msg = f"{what}: {status_string(status)} ({status})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


class SpmvArgError(SpmvError, ValueError):
    """An argument the binding refuses before calling the library: a tensor
    that is not on the GPU, not contiguous, of the wrong element type or too
    short for what the call will read or write (status SPMV_E_ARG)."""

    def __init__(self, what: str, detail: str):
        self.status = SPMV_E_ARG
        ValueError.__init__(self, f"{what}: invalid argument: {detail}")


class spmv_stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("sum_len", ctypes.c_int64),
                ("sum_len2", ctypes.c_int64), ("max_row", ctypes.c_int32), ("min_row", ctypes.c_int32),
                ("max_col", ctypes.c_int32), ("bandwidth", ctypes.c_int32), ("mu", ctypes.c_double),
                ("sigma", ctypes.c_double),
                ("d_mat", ctypes.c_double)]


class spmv_sizes(ctypes.Structure):
    _fields_ = [("bytes", ctypes.c_size_t * 4), ("workspace", ctypes.c_size_t), ("width", ctypes.c_int32)]


class spmv_buffers(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p * 4), ("bytes", ctypes.c_size_t * 4)]


class at_table(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("d_star", ctypes.c_double), ("calibrated", ctypes.c_int32),
                ("spmv_bps", (((ctypes.c_double * AT_DBUCKETS) * 2) * 6) * 2),
                ("trans_bps", ((ctypes.c_double * AT_DBUCKETS) * 6) * 2), ("launch_s", ctypes.c_double),
                ("k_margin", ctypes.c_double)]


class spmv_server_config(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("policy", ctypes.c_int32), ("hbm_cap", ctypes.c_size_t),
                ("table", at_table)]


class spmv_job(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("arrival_s", ctypes.c_double), ("n", ctypes.c_int32),
                ("nnz", ctypes.c_int64), ("irp", ctypes.c_void_p), ("icol", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("x0", ctypes.c_void_p), ("k", ctypes.c_int32),
                ("shift", ctypes.c_int32), ("y_out", ctypes.c_void_p)]


class spmv_job_result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int32), ("format", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("arrival_s", ctypes.c_double), ("admit_s", ctypes.c_double),
                ("ready_s", ctypes.c_double), ("done_s", ctypes.c_double), ("d_mat", ctypes.c_double),
                ("device_bytes", ctypes.c_size_t)]


class at_decision(ctypes.Structure):
    _fields_ = [("rule", ctypes.c_int32), ("feasible_ell", ctypes.c_int32), ("d_mat", ctypes.c_double),
                ("t_crs_hat", ctypes.c_double), ("t_fmt_hat", ctypes.c_double),
                ("t_trans_hat", ctypes.c_double), ("k_break_even", ctypes.c_double)]


def build() -> None:
    """Compile libspmvat.so for gfx950 in place (always recompiles)."""
    subprocess.run(["make", "-B", "-s", "-j8", "-C", os.path.join(_HERE, "csrc")], check=True)


def lib():
    """The loaded library; raises when it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libspmvat.so is not built ({LIB_PATH}); run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, sz, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
        st = ctypes.c_int
        L.spmv_plan_workspace_bytes.argtypes = [i32, i64]
        L.spmv_plan_workspace_bytes.restype = sz
        L.spmv_plan_create.argtypes = [ctypes.POINTER(P), i32, i64, P, P, P, ctypes.c_int, P, sz, P]
        L.spmv_plan_create.restype = st
        L.spmv_plan_stats.argtypes = [P, ctypes.POINTER(spmv_stats)]
        L.spmv_plan_stats.restype = st
        L.spmv_plan_value_type.argtypes = [P, ctypes.POINTER(ctypes.c_int)]
        L.spmv_plan_value_type.restype = st
        L.spmv_plan_set_limit.argtypes = [P, sz]
        L.spmv_plan_set_limit.restype = st
        L.spmv_plan_set_ccs_algorithm.argtypes = [P, ctypes.c_int]
        L.spmv_plan_set_ccs_algorithm.restype = st
        L.spmv_buffer_sizes.argtypes = [P, ctypes.c_int, ctypes.POINTER(spmv_sizes)]
        L.spmv_buffer_sizes.restype = st
        for name in ("csr_to_coo", "csr_to_ell"):
            fn = getattr(L, name)
            fn.argtypes = [P, ctypes.c_int, ctypes.POINTER(spmv_buffers), P, sz, P]
            fn.restype = st
        L.csr_to_ccs.argtypes = [P, ctypes.POINTER(spmv_buffers), P, sz, P]
        L.csr_to_ccs.restype = st
        L.spmv_ccs_inplace_workspace_bytes.argtypes = [P, ctypes.POINTER(sz)]
        L.spmv_ccs_inplace_workspace_bytes.restype = st
        L.csr_to_ccs_inplace.argtypes = [P, P, P, P, P, sz, P]
        L.csr_to_ccs_inplace.restype = st
        L.spmv_exec.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P, P]
        L.spmv_exec.restype = st
        L.spmv_exec_coo_row_noalloc.argtypes = [i32, i64, P, P, P, ctypes.c_int, P, P, P]
        L.spmv_exec_coo_row_noalloc.restype = st
        L.at_table_build.argtypes = [P, P, P, i32, f64, ctypes.POINTER(at_table)]
        L.at_table_build.restype = st
        L.at_choose_format.argtypes = [P, ctypes.POINTER(at_table), i64, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(at_decision)]
        L.at_choose_format.restype = st
        L.at_choose_format_stats.argtypes = [ctypes.POINTER(spmv_stats), ctypes.c_int, sz, ctypes.POINTER(at_table),
                                             i64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                             ctypes.POINTER(at_decision)]
        L.at_choose_format_stats.restype = st
        L.spmv_convert_values.argtypes = [P, P, i64, ctypes.c_int, P]
        L.spmv_convert_values.restype = st
        L.spmv_plan_destroy.argtypes = [P]
        L.spmv_plan_destroy.restype = None
        L.spmv_status_string.argtypes = [ctypes.c_int]
        L.spmv_status_string.restype = ctypes.c_char_p
        L.spmv_plan_last_error.argtypes = [P]
        L.spmv_plan_last_error.restype = ctypes.c_char_p
        L.spmv_server_create.argtypes = [ctypes.POINTER(spmv_server_config), ctypes.POINTER(P)]
        L.spmv_server_create.restype = st
        L.spmv_server_start.argtypes = [P]
        L.spmv_server_start.restype = st
        L.spmv_server_submit.argtypes = [P, ctypes.POINTER(spmv_job)]
        L.spmv_server_submit.restype = st
        L.spmv_server_wait.argtypes = [P, f64]
        L.spmv_server_wait.restype = st
        L.spmv_server_results.argtypes = [P, ctypes.POINTER(spmv_job_result), i32]
        L.spmv_server_results.restype = i32
        L.spmv_server_destroy.argtypes = [P]
        L.spmv_server_destroy.restype = None
        L.spmv_arena_create.argtypes = [sz]
        L.spmv_arena_create.restype = P
        L.spmv_arena_alloc.argtypes = [P, sz]
        L.spmv_arena_alloc.restype = i64
        L.spmv_arena_free.argtypes = [P, i64, sz]
        L.spmv_arena_free.restype = None
        L.spmv_arena_free_bytes.argtypes = [P]
        L.spmv_arena_free_bytes.restype = sz
        L.spmv_arena_largest.argtypes = [P]
        L.spmv_arena_largest.restype = sz
        L.spmv_arena_destroy.argtypes = [P]
        L.spmv_arena_destroy.restype = None
        _LIB = L
    return _LIB


# ------------------------------------------------------------- marshalling

def _ptr(t) -> ctypes.c_void_p:
    if t is None:
        return ctypes.c_void_p(None)
    if isinstance(t, int):
        return ctypes.c_void_p(t)
    return ctypes.c_void_p(t.data_ptr() if t.numel() > 0 else None)


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(stream)


def _check(status: int, what: str, plan=None) -> None:
    if status != SPMV_OK:
        detail = ""
        if plan is not None and status == SPMV_E_HIP:
            detail = lib().spmv_plan_last_error(plan).decode()
        raise SpmvError(status, what, detail)


def _dev(t, what: str, name: str, dtype=None, numel: int = 0, device=None):
    """Checks that t (a torch tensor handed to the library as a device
    pointer) lives on the GPU, is contiguous, has element type `dtype` (when
    given) and holds at least `numel` elements.  Raw integer addresses pass
    unchecked: they are the C ABI's own contract.  Marshalling only."""
    if t is None or isinstance(t, int):
        return
    if not isinstance(t, torch.Tensor):
        raise SpmvArgError(what, f"{name} must be a torch tensor, not {type(t).__name__}")
    if not t.is_cuda:
        raise SpmvArgError(what, f"{name} must be a GPU tensor (it is on {t.device})")
    if device is not None and t.device != device:
        raise SpmvArgError(what, f"{name} is on {t.device}, the other arrays on {device}")
    if not t.is_contiguous():
        raise SpmvArgError(what, f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise SpmvArgError(what, f"{name} must be {dtype}, not {t.dtype}")
    if t.numel() < numel:
        raise SpmvArgError(what, f"{name} holds {t.numel()} elements, needs at least {numel}")


def _overlap(a, b) -> bool:
    """Whether the storage of two tensors overlaps (both on the GPU)."""
    if not isinstance(a, torch.Tensor) or not isinstance(b, torch.Tensor) or a.numel() == 0 or b.numel() == 0:
        return False
    a0, b0 = a.data_ptr(), b.data_ptr()
    return a0 < b0 + b.numel() * b.element_size() and b0 < a0 + a.numel() * a.element_size()


def vector_dtype(val_type: int) -> torch.dtype:
    """Element type of x and y for a plan whose values are stored as
    val_type: binary64 with binary64 values, else binary32."""
    return torch.float64 if val_type == F64 else torch.float32


def status_string(s: int) -> str:
    return lib().spmv_status_string(s).decode()


def _buffers(tensors, what: str = "buffers") -> spmv_buffers:
    b = spmv_buffers()
    for k, t in enumerate(tensors):
        _dev(t, what, f"out[{k}]")
        b.ptr[k] = _ptr(t).value
        b.bytes[k] = t.numel() * t.element_size()
    return b


# --------------------------------------------------- the C ABI, by name

def spmv_plan_workspace_bytes(n: int, nnz: int) -> int:
    return int(lib().spmv_plan_workspace_bytes(n, nnz))


def spmv_plan_create(n, nnz, irp, icol, val, val_type, plan_work, stream=None) -> ctypes.c_void_p:
    w = "spmv_plan_create"
    if val_type not in TORCH_OF_DTYPE:
        raise SpmvArgError(w, f"unknown value type {val_type}")
    dev = irp.device if isinstance(irp, torch.Tensor) else None
    _dev(irp, w, "irp", torch.int32, n + 1)
    _dev(icol, w, "icol", torch.int32, nnz, dev)
    _dev(val, w, "val", TORCH_OF_DTYPE[val_type], nnz, dev)
    _dev(plan_work, w, "plan_work", None, 0, dev)
    h = ctypes.c_void_p()
    s = lib().spmv_plan_create(ctypes.byref(h), n, nnz, _ptr(irp), _ptr(icol), _ptr(val), val_type,
                               _ptr(plan_work), plan_work.numel() * plan_work.element_size(), _stream(stream))
    _check(s, "spmv_plan_create")
    return h


def spmv_plan_stats(plan) -> spmv_stats:
    out = spmv_stats()
    _check(lib().spmv_plan_stats(plan, ctypes.byref(out)), "spmv_plan_stats")
    return out


def spmv_plan_set_limit(plan, max_format_bytes: int) -> None:
    _check(lib().spmv_plan_set_limit(plan, max_format_bytes), "spmv_plan_set_limit")


def spmv_plan_set_ccs_algorithm(plan, alg: int) -> None:
    _check(lib().spmv_plan_set_ccs_algorithm(plan, alg), "spmv_plan_set_ccs_algorithm")


def spmv_buffer_sizes(plan, fmt: int):
    """(status, spmv_sizes): sizes are filled even for SPMV_E_TOO_LARGE."""
    out = spmv_sizes()
    s = lib().spmv_buffer_sizes(plan, fmt, ctypes.byref(out))
    return s, out


def csr_to_coo(plan, column_wise: int, out, work=None, stream=None) -> None:
    b = _buffers(out, "csr_to_coo")
    _dev(work, "csr_to_coo", "work")
    wb = 0 if work is None else work.numel() * work.element_size()
    _check(lib().csr_to_coo(plan, column_wise, ctypes.byref(b), _ptr(work), wb, _stream(stream)), "csr_to_coo", plan)


def csr_to_ccs(plan, out, work, stream=None) -> None:
    b = _buffers(out, "csr_to_ccs")
    _dev(work, "csr_to_ccs", "work")
    wb = work.numel() * work.element_size()
    _check(lib().csr_to_ccs(plan, ctypes.byref(b), _ptr(work), wb, _stream(stream)), "csr_to_ccs", plan)


def spmv_ccs_inplace_workspace_bytes(plan) -> int:
    out = ctypes.c_size_t()
    _check(lib().spmv_ccs_inplace_workspace_bytes(plan, ctypes.byref(out)), "spmv_ccs_inplace_workspace_bytes")
    return out.value


def csr_to_ccs_inplace(plan, irp, icol, val, work, stream=None) -> None:
    w = "csr_to_ccs_inplace"
    _dev(irp, w, "irp", torch.int32)
    _dev(icol, w, "icol", torch.int32)
    _dev(val, w, "val")
    _dev(work, w, "work")
    wb = work.numel() * work.element_size()
    _check(lib().csr_to_ccs_inplace(plan, _ptr(irp), _ptr(icol), _ptr(val), _ptr(work), wb, _stream(stream)), w,
           plan)


def csr_to_ell(plan, column_wise: int, out, work=None, stream=None) -> None:
    b = _buffers(out, "csr_to_ell")
    _dev(work, "csr_to_ell", "work")
    wb = 0 if work is None else work.numel() * work.element_size()
    _check(lib().csr_to_ell(plan, column_wise, ctypes.byref(b), _ptr(work), wb, _stream(stream)), "csr_to_ell", plan)


def spmv_plan_value_type(plan) -> int:
    out = ctypes.c_int()
    _check(lib().spmv_plan_value_type(plan, ctypes.byref(out)), "spmv_plan_value_type")
    return out.value


def spmv_exec(plan, fmt: int, variant: int, x, y, stream=None) -> None:
    if isinstance(x, torch.Tensor) or isinstance(y, torch.Tensor):
        w = "spmv_exec"
        n = spmv_plan_stats(plan).n
        vt = vector_dtype(spmv_plan_value_type(plan))
        _dev(x, w, "x", vt, n)
        _dev(y, w, "y", vt, n, x.device if isinstance(x, torch.Tensor) else None)
        if _overlap(x, y):
            raise SpmvArgError(w, "x and y must not overlap")
    _check(lib().spmv_exec(plan, fmt, variant, _ptr(x), _ptr(y), _stream(stream)), "spmv_exec", plan)


COO_ROW_NOALLOC_MAX_NNZ = 134217728   # SPMV_COO_ROW_NOALLOC_MAX_NNZ


def spmv_exec_coo_row_noalloc(n: int, nnz: int, irow, icol, val, val_type: int, x, y, stream=None) -> None:
    """y = A x in COO-Row form with no plan and no workspace (the library's
    fixed per-device array holds the carries).  Same checks as spmv_exec."""
    w = "spmv_exec_coo_row_noalloc"
    if val_type not in TORCH_OF_DTYPE:
        raise SpmvArgError(w, f"unknown value type {val_type}")
    dev = x.device if isinstance(x, torch.Tensor) else None
    _dev(irow, w, "irow", torch.int32, nnz, dev)
    _dev(icol, w, "icol", torch.int32, nnz, dev)
    _dev(val, w, "val", TORCH_OF_DTYPE[val_type], nnz, dev)
    vt = vector_dtype(val_type)
    _dev(x, w, "x", vt, n)
    _dev(y, w, "y", vt, n, dev)
    if _overlap(x, y):
        raise SpmvArgError(w, "x and y must not overlap")
    _check(lib().spmv_exec_coo_row_noalloc(n, nnz, _ptr(irow), _ptr(icol), _ptr(val), val_type, _ptr(x), _ptr(y),
                                           _stream(stream)), w)


def at_table_build(d, r, feasible=None, c: float = 1.0) -> at_table:
    m = len(d)
    D = (ctypes.c_double * max(m, 1))(*d)
    R = (ctypes.c_double * max(m, 1))(*r)
    F = (ctypes.c_int32 * max(m, 1))(*(feasible if feasible is not None else [1] * m))
    out = at_table()
    _check(lib().at_table_build(D, R, F, m, c, ctypes.byref(out)), "at_table_build")
    return out


def at_choose_format(plan, table: at_table, k_repeats: int):
    """(format, variant, at_decision)."""
    f, v, why = ctypes.c_int(), ctypes.c_int(), at_decision()
    _check(lib().at_choose_format(plan, ctypes.byref(table), k_repeats, ctypes.byref(f), ctypes.byref(v),
                                  ctypes.byref(why)), "at_choose_format")
    return f.value, v.value, why


def at_choose_format_stats(stats: spmv_stats, val_type: int, max_format_bytes: int, table: at_table,
                           k_repeats: int):
    """(format, variant, at_decision) from statistics alone (host only)."""
    f, v, why = ctypes.c_int(), ctypes.c_int(), at_decision()
    _check(lib().at_choose_format_stats(ctypes.byref(stats), val_type, max_format_bytes, ctypes.byref(table),
                                        k_repeats, ctypes.byref(f), ctypes.byref(v), ctypes.byref(why)),
           "at_choose_format_stats")
    return f.value, v.value, why


def spmv_convert_values(inp, out, to: int, stream=None) -> None:
    w = "spmv_convert_values"
    if to not in (F32, BF16, F16):
        raise SpmvArgError(w, f"target type must be F32, BF16 or F16, not {to}")
    _dev(inp, w, "in", torch.float64)
    _dev(out, w, "out", TORCH_OF_DTYPE[to], inp.numel(), inp.device)
    _check(lib().spmv_convert_values(_ptr(inp), _ptr(out), inp.numel(), to, _stream(stream)), "spmv_convert_values")


def spmv_plan_destroy(plan) -> None:
    lib().spmv_plan_destroy(plan)


def spmv_server_create(cfg: spmv_server_config) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().spmv_server_create(ctypes.byref(cfg), ctypes.byref(h)), "spmv_server_create")
    return h


def spmv_server_start(srv) -> None:
    _check(lib().spmv_server_start(srv), "spmv_server_start")


def spmv_server_submit(srv, job: spmv_job) -> None:
    _check(lib().spmv_server_submit(srv, ctypes.byref(job)), "spmv_server_submit")


def spmv_server_wait(srv, timeout_s: float) -> int:
    return lib().spmv_server_wait(srv, timeout_s)


def spmv_server_results(srv, cap: int):
    out = (spmv_job_result * max(cap, 1))()
    m = lib().spmv_server_results(srv, out, cap)
    return [out[i] for i in range(m)]


def spmv_server_destroy(srv) -> None:
    lib().spmv_server_destroy(srv)


# ---------------------------------------------------------- convenience

def at_table_from_json(d: dict) -> at_table:
    """An at_table from the off-line phase's JSON (see offline.py)."""
    t = at_table_build(d.get("d", []), d.get("r", []), d.get("feasible"), d.get("c", 1.0))
    cm = d.get("cost_model")
    if cm:
        if not isinstance(cm.get("spmv_bps"), list) or len(cm["spmv_bps"]) != 2:
            raise ValueError("cost_model must hold one entry per locality class (local, scattered); "
                             "re-run the off-line phase")
        t.calibrated = 1
        for loc, per_f in enumerate(cm["spmv_bps"]):
            for f_, per_v in per_f.items():
                for v_, buckets in enumerate(per_v):
                    for b_, val in enumerate(buckets):
                        t.spmv_bps[loc][int(f_)][v_][b_] = val
        for loc, per_f in enumerate(cm["trans_bps"]):
            for f_, buckets in per_f.items():
                for b_, val in enumerate(buckets):
                    t.trans_bps[loc][int(f_)][b_] = val
        t.launch_s = cm.get("launch_s", 0.0)
    t.k_margin = float(d.get("k_margin", 0.0) or 0.0)
    return t


# Sources of the kernels the off-line phase times (row statistics, the COO
# and ELL transformations, the CRS / COO-Row / ELL-Row SpMVs and the serving
# step it calibrates the margin on): the auto-tuning table depends on these
# only.
TABLE_KERNEL_SOURCES = ("common.h", "spmv_rows.h", "k_stats.hip", "k_transform.hip", "k_spmv.hip", "k_serve.hip")


def kernel_source_sha(files=None) -> str:
    """Hash of kernel sources: by default every csrc/*.hip and *.h but the
    header of the host-only code; else the named files of csrc.  A table or
    profile measured with other kernels carries another value."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(_HERE, "csrc")
    names = sorted(files) if files is not None else \
        [f for f in sorted(os.listdir(d)) if f.endswith((".hip", ".h")) and f != "host_core.h"]
    for f in names:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def table_kernel_sha() -> str:
    """Hash of the sources of the kernels the off-line table is measured on."""
    return kernel_source_sha(TABLE_KERNEL_SOURCES)


def table_matches_kernels(d: dict):
    """Whether an off-line table (its JSON) was measured with this tree's
    kernels of the off-line phase: True / False, or None when the table
    carries no stamp."""
    sha = d.get("kernel_source_sha")
    return None if sha is None else sha == table_kernel_sha()


def convert_values(val64: torch.Tensor, to: int, stream=None) -> torch.Tensor:
    """binary64 device values -> a new tensor of the storage type `to`."""
    out = torch.empty(val64.numel(), dtype=TORCH_OF_DTYPE[to], device=val64.device)
    spmv_convert_values(val64, out, to, stream)
    return out


class Plan:
    """Owns a plan over device CRS arrays and the device buffers of every
    format built on it (torch tensors, kept alive with the plan)."""

    def __init__(self, irp: torch.Tensor, icol: torch.Tensor, val: torch.Tensor, stream=None):
        if val.dtype not in DTYPE_OF_TORCH:
            raise SpmvArgError("Plan", f"val must be float64, float32, bfloat16 or float16, not {val.dtype}")
        _dev(irp, "Plan", "irp", torch.int32, 1)
        _dev(icol, "Plan", "icol", torch.int32, 0, irp.device)
        _dev(val, "Plan", "val", val.dtype, icol.numel(), irp.device)
        self.n = irp.numel() - 1
        self.nnz = icol.numel()
        self.dtype = DTYPE_OF_TORCH[val.dtype]
        self.device = irp.device
        self.crs = (irp, icol, val)
        self.work = torch.empty(spmv_plan_workspace_bytes(self.n, self.nnz), dtype=torch.uint8, device=self.device)
        self.handle = spmv_plan_create(self.n, self.nnz, irp, icol, val, self.dtype, self.work, stream)
        self.buffers = {}
        self.ccs_work = None

    def __del__(self):
        self.close()

    def close(self) -> None:
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            spmv_plan_destroy(h)
            self.handle = None

    @property
    def stats(self) -> spmv_stats:
        return spmv_plan_stats(self.handle)

    def set_limit(self, max_format_bytes: int) -> None:
        spmv_plan_set_limit(self.handle, max_format_bytes)

    def sizes(self, fmt: int):
        return spmv_buffer_sizes(self.handle, fmt)

    def _alloc(self, fmt: int):
        s, sz = self.sizes(fmt)
        _check(s, f"spmv_buffer_sizes({FORMAT_NAMES[fmt]})")
        vt = TORCH_OF_DTYPE[self.dtype]
        vb = torch.empty(0, dtype=vt).element_size()
        dev = self.device
        if fmt in (COO_ROW, COO_COL):
            out = [torch.empty(sz.bytes[0] // 4, dtype=torch.int32, device=dev)]
        elif fmt == CCS:
            out = [torch.empty(sz.bytes[0] // 4, dtype=torch.int32, device=dev),
                   torch.empty(sz.bytes[1] // 4, dtype=torch.int32, device=dev),
                   torch.empty(sz.bytes[2] // vb, dtype=vt, device=dev)]
        else:
            out = [torch.empty(sz.bytes[0] // vb, dtype=vt, device=dev),
                   torch.empty(sz.bytes[1] // 4, dtype=torch.int32, device=dev)]
        work = torch.empty(sz.workspace, dtype=torch.uint8, device=dev) if sz.workspace else None
        return out, work, sz

    def to_coo(self, column_wise: bool = False, stream=None):
        fmt = COO_COL if column_wise else COO_ROW
        out, _, _ = self._alloc(fmt)
        csr_to_coo(self.handle, int(column_wise), out, None, stream)
        self.buffers[fmt] = out
        return out

    def to_ccs(self, stream=None, algorithm: int | None = None):
        if algorithm is not None:
            spmv_plan_set_ccs_algorithm(self.handle, algorithm)
        out, work, _ = self._alloc(CCS)
        csr_to_ccs(self.handle, out, work, stream)
        self.buffers[CCS] = out
        self.ccs_work = work
        for f in (COO_COL, ELL_COL):
            self.buffers.pop(f, None)
        return out

    def to_ccs_inplace(self, stream=None):
        """CCS over the plan's own CRS tensors (the copy-back of Phase I):
        afterwards irp, icol and val hold the column pointers, row numbers
        and values, and CRS-based calls return SPMV_E_NOT_READY."""
        irp, icol, val = self.crs
        work = torch.empty(max(spmv_ccs_inplace_workspace_bytes(self.handle), 16), dtype=torch.uint8,
                           device=self.device)
        csr_to_ccs_inplace(self.handle, irp, icol, val, work, stream)
        for f in (COO_ROW, CCS, COO_COL, ELL_COL):
            self.buffers.pop(f, None)
        self.buffers[CCS] = [irp, icol, val]
        self.inplace_work = work    # kept until the stream has used it
        return irp, icol, val

    def to_ell(self, column_wise: bool = False, stream=None):
        fmt = ELL_COL if column_wise else ELL_ROW
        out, _, sz = self._alloc(fmt)
        csr_to_ell(self.handle, int(column_wise), out, None, stream)
        self.buffers[fmt] = out
        return out, sz.width

    def release(self, fmt: int) -> None:
        self.buffers.pop(fmt, None)

    def spmv(self, fmt: int, x: torch.Tensor, y: torch.Tensor | None = None, variant: int = 0, stream=None):
        if y is None:
            y = torch.empty_like(x)
        spmv_exec(self.handle, fmt, variant, x, y, stream)
        return y

    def choose(self, table: at_table, k_repeats: int = 0):
        return at_choose_format(self.handle, table, k_repeats)

