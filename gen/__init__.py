"""Seeded synthetic workloads: CRS matrices and x vectors.

This module only builds inputs.  It holds no arithmetic of the method (no
transformation, SpMV or D_mat): the CPU oracle and the GPU library both take
their inputs from here and nothing else is shared between them.

Arrays follow the paper's CRS definition (section 2.1) shifted to 0-based:
``irp[n+1]`` (row pointers, irp[0] = 0, irp[n] = nnz), ``icol[nnz]`` and
``val[nnz]`` (FP64).  Every draw is counter based (SplitMix64 over
(seed, stream, counter)), so results do not depend on thread counts.
"""
from __future__ import annotations

import ctypes
import json
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

BASE_SEED = 20240700019
ST_X = 1


def build() -> None:
    """Compile libspmvgen.so in place (always recompiles)."""
    subprocess.run(["make", "-B", "-s", "-C", _HERE], check=True)


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libspmvgen.so")
        if not os.path.exists(path):
            build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64, u64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        lib.gen_uniform.argtypes = [i64, f64, f64, u64, u64, P]
        lib.gen_normal.argtypes = [i64, u64, u64, P]
        lib.gen_lap2d.argtypes = [i32, i32, f64, f64, P, P, P]
        lib.gen_lap2d.restype = i64
        lib.gen_stencil27.argtypes = [i32, i32, i32, ctypes.c_int, u64, P, P, P]
        lib.gen_stencil27.restype = i64
        lib.gen_lognormal_lengths.argtypes = [i32, f64, f64, i32, i32, u64, P]
        lib.gen_lengths_to_irp.argtypes = [i32, P, P]
        lib.gen_lengths_to_irp.restype = i64
        lib.gen_random_cols.argtypes = [i32, i32, P, u64, P]
        lib.gen_window_cols.argtypes = [i32, i32, P, u64, P]
        lib.gen_banded.argtypes = [i32, i32, u64, P, P, P]
        lib.gen_banded.restype = i64
        lib.gen_unif_stream.argtypes = [i64, u64, u64, P]
        _LIB = lib
    return _LIB


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


@dataclass
class Crs:
    """A square CRS matrix held in host memory (0-based, int32 indices)."""
    n: int
    irp: np.ndarray
    icol: np.ndarray
    val: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.icol.shape[0])


# ------------------------------------------------------------------ vectors

def x_uniform(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    _lib().gen_uniform(n, lo, hi, seed, ST_X, _p(out))
    return out


def normal(m: int, seed: int, stream: int = 2) -> np.ndarray:
    out = np.empty(m, dtype=np.float64)
    _lib().gen_normal(m, seed, stream, _p(out))
    return out


def unif_stream(m: int, seed: int, stream: int) -> np.ndarray:
    out = np.empty(m, dtype=np.float64)
    _lib().gen_unif_stream(m, seed, stream, _p(out))
    return out


# ----------------------------------------------------------------- matrices

def lap2d(nx: int, ny: int, diag: float = 4.0, off: float = -1.0) -> Crs:
    lib = _lib()
    nnz = lib.gen_lap2d(nx, ny, diag, off, None, None, None)
    n = nx * ny
    irp = np.empty(n + 1, np.int32)
    icol = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    lib.gen_lap2d(nx, ny, diag, off, _p(irp), _p(icol), _p(val))
    return Crs(n, irp, icol, val, f"lap2d_{nx}x{ny}")


def stencil27(nx: int, ny: int, nz: int, seed: int, integer_values: bool = False) -> Crs:
    lib = _lib()
    nnz = lib.gen_stencil27(nx, ny, nz, int(integer_values), seed, None, None, None)
    n = nx * ny * nz
    irp = np.empty(n + 1, np.int32)
    icol = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    lib.gen_stencil27(nx, ny, nz, int(integer_values), seed, _p(irp), _p(icol), _p(val))
    return Crs(n, irp, icol, val, f"stencil27_{nx}x{ny}x{nz}")


def lognormal_lengths(n: int, mean: float, s: float, lmin: int, lmax: int, seed: int) -> np.ndarray:
    out = np.empty(n, np.int32)
    _lib().gen_lognormal_lengths(n, mean, s, lmin, lmax, seed, _p(out))
    return out


def random_rows(n: int, lengths: np.ndarray, seed: int) -> Crs:
    """Rows with the given lengths, columns uniform without replacement and
    sorted, values N(0,1)."""
    lib = _lib()
    lengths = np.ascontiguousarray(lengths, dtype=np.int32)
    irp = np.empty(n + 1, np.int32)
    nnz = lib.gen_lengths_to_irp(n, _p(lengths), _p(irp))
    if nnz < 0:
        raise ValueError("nnz exceeds the int32 range")
    icol = np.empty(nnz, np.int32)
    lib.gen_random_cols(n, n, _p(irp), seed, _p(icol))
    val = normal(nnz, seed)
    return Crs(n, irp, icol, val)


def window_rows(n: int, lengths: np.ndarray, window: int, seed: int) -> Crs:
    """Rows with the given lengths, columns uniform without replacement from
    [i - window, i + window] (clipped), sorted; values N(0,1)."""
    lib = _lib()
    lengths = np.ascontiguousarray(lengths, dtype=np.int32)
    idx = np.arange(n)
    room = (np.minimum(idx + window, n - 1) - np.maximum(idx - window, 0) + 1).astype(np.int32)
    if np.any(lengths > room):
        raise ValueError("a row is longer than its column window")
    irp = np.empty(n + 1, np.int32)
    nnz = lib.gen_lengths_to_irp(n, _p(lengths), _p(irp))
    if nnz < 0:
        raise ValueError("nnz exceeds the int32 range")
    icol = np.empty(nnz, np.int32)
    lib.gen_window_cols(n, window, _p(irp), seed, _p(icol))
    val = normal(nnz, seed)
    return Crs(n, irp, icol, val)


def lognormal_matrix(n: int, mean: float, s: float, seed: int, lmin: int = 1, lmax: int = 8192) -> Crs:
    m = random_rows(n, lognormal_lengths(n, mean, s, lmin, lmax, seed), seed)
    m.name = f"lognormal_n{n}_m{mean:g}_s{s:g}"
    return m


def banded(n: int, b: int, seed: int) -> Crs:
    lib = _lib()
    nnz = lib.gen_banded(n, b, seed, None, None, None)
    irp = np.empty(n + 1, np.int32)
    icol = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    lib.gen_banded(n, b, seed, _p(irp), _p(icol), _p(val))
    return Crs(n, irp, icol, val, f"banded_n{n}_b{b}")


def random_small(n: int, seed: int, max_len: int = 8, sorted_rows: bool = True,
                 duplicates: bool = False, empty_frac: float = 0.2,
                 integer_values: bool = True) -> Crs:
    """Tiny random pattern for brute-force tests.  May contain empty rows,
    unsorted rows and duplicate (row, col) entries when asked to."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, max_len + 1, size=n)
    lens[rng.random(n) < empty_frac] = 0
    irp = np.zeros(n + 1, np.int64)
    irp[1:] = np.cumsum(lens)
    cols = []
    for i in range(n):
        k = int(lens[i])
        if duplicates:
            c = rng.integers(0, n, size=k)
        else:
            c = rng.choice(n, size=min(k, n), replace=False)
            if len(c) < k:
                c = np.concatenate([c, rng.integers(0, n, size=k - len(c))])
        if sorted_rows:
            c = np.sort(c)
        cols.append(c)
    icol = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    irp = irp.astype(np.int32)
    if integer_values:
        val = rng.integers(-4, 5, size=icol.shape[0]).astype(np.float64)
    else:
        val = rng.standard_normal(icol.shape[0])
    return Crs(n, irp, icol, val, f"small_n{n}_s{seed}")


# ------------------------------------------------------------ the workloads

def seed_for(config: int, index: int = 0) -> int:
    return BASE_SEED + config * 1000 + index


def laplace_64x64() -> Crs:
    """2-D 5-point Laplacian on a 64x64 grid: n = 4096, nnz = 20224,
    4.0 on the diagonal and -1.0 off it."""
    return lap2d(64, 64)


def stencil27_128(integer_values: bool = False, edge: int = 128) -> Crs:
    """27-point stencil on an edge^3 grid with Dirichlet truncation
    (edge = 128: n = 2,097,152, nnz = 382^3 = 55,742,968)."""
    return stencil27(edge, edge, edge, seed_for(2), integer_values)


POWERLAW_N = 4_194_304


def powerlaw(n: int = POWERLAW_N) -> Crs:
    """Row lengths round(LogNormal) with mean 16 and log-sigma 1.2, clipped to
    [1, 8192]; columns uniform without replacement; values N(0,1)."""
    m = lognormal_matrix(n, 16.0, 1.2, seed_for(3))
    m.name = f"powerlaw_n{n}"
    return m


DSWEEP_N = 1_048_576
DSWEEP_TARGETS = [0.125 * k for k in range(33)]


def dsweep_table() -> dict:
    """Log-sigma per D_mat target of the row-length sweep (input recipe,
    written by tests/golden/make_dsweep_table.py)."""
    with open(os.path.join(_HERE, "dsweep_s.json")) as f:
        return json.load(f)


def dsweep_lengths(s: float, n: int = DSWEEP_N) -> np.ndarray:
    """Row lengths of the sweep: round(exp(ln 32 - s^2/2 + s z_i)) clipped to
    [1, 8192], one shared seeded z vector across the whole sweep."""
    return lognormal_lengths(n, 32.0, s, 1, 8192, seed_for(5))


DSWEEP_WINDOW = 4096


def dsweep_matrix(index: int, n: int = DSWEEP_N, local: bool = False) -> Crs:
    """Sweep matrix `index`: uniform columns over the whole row (default) or
    over the window [i - 4096, i + 4096] around the row (local=True, the
    banded-structure family; lengths clipped to the window)."""
    tab = dsweep_table()
    s = float(tab["s"][index])
    lens = dsweep_lengths(s, n)
    if local:
        idx = np.arange(n)
        room = np.minimum(idx + DSWEEP_WINDOW, n - 1) - np.maximum(idx - DSWEEP_WINDOW, 0) + 1
        lens = np.minimum(lens, room).astype(np.int32)
        m = window_rows(n, lens, DSWEEP_WINDOW, seed_for(5, 500 + index))
    else:
        m = random_rows(n, lens, seed_for(5, index))
    m.name = f"dsweep{'_local' if local else ''}_{index}_D{DSWEEP_TARGETS[index]:.3f}"
    return m


# Stand-ins for the paper's test matrices (section 4.2, Table 1): each has
# the printed N, mean row length and D_mat (nnz follows from N and the mean,
# within a few percent), columns uniform within 4096 of the diagonal (the
# printed matrices are near-banded FEM and circuit matrices; their column
# structure is not printed).  The lognormal log-sigma per matrix is the input
# recipe written by tests/golden/make_table1_standins.py.
TABLE1_WINDOW = 4096


def table1_lengths(n: int, mean: float, s: float, seed: int) -> np.ndarray:
    """Row lengths round(exp(ln mean - s^2/2 + s z_i)) clipped to [1, 8193]
    and to the row's column window."""
    lens = lognormal_lengths(n, mean, s, 1, min(n, 2 * TABLE1_WINDOW + 1), seed)
    idx = np.arange(n)
    room = np.minimum(idx + TABLE1_WINDOW, n - 1) - np.maximum(idx - TABLE1_WINDOW, 0) + 1
    return np.minimum(lens, room).astype(np.int32)


def table1_recipe() -> dict:
    with open(os.path.join(_HERE, "table1_s.json")) as f:
        return json.load(f)


def table1_standin(no: int) -> Crs:
    """Stand-in for Table 1 matrix number `no` (1..22)."""
    tab = table1_recipe()
    k = tab["no"].index(no)
    n, mean, s = tab["n"][k], tab["mu"][k], tab["s"][k]
    lens = table1_lengths(n, mean, s, seed_for(6, no))
    m = window_rows(n, lens, TABLE1_WINDOW, seed_for(6, 100 + no))
    m.name = f"table1_{no}_{tab['name'][k]}"
    return m


@dataclass
class Job:
    """One SpMV job of the serving stream."""
    index: int
    arrival_s: float
    k: int
    kind: str          # "banded" or "random"
    n: int
    band: int = 0
    mean: float = 0.0
    s: float = 0.0

    def matrix(self) -> Crs:
        seed = seed_for(4, self.index)
        if self.kind == "banded":
            m = banded(self.n, self.band, seed)
        else:
            m = lognormal_matrix(self.n, self.mean, self.s, seed, 1, min(8192, self.n))
        # values are stored in FP32 from generation on
        m.val = m.val.astype(np.float32).astype(np.float64)
        m.name = f"job{self.index}_{self.kind}_n{self.n}"
        return m


def serving_jobs(count: int = 2048, rate_per_s: float = 2000.0, n_max: float = 5e5) -> list:
    """Poisson arrivals (rate_per_s; 0 means all at t = 0), n log-uniform in
    [1e3, n_max], structure alternating banded (half-bandwidth
    round(exp U[0, ln 64])) and lognormal random rows (mean exp U[ln 8, ln 64],
    log-sigma U[0.1, 1.2]), repeat count k = round(exp U[0, ln 500])."""
    seed = seed_for(4)
    u = unif_stream(8 * count, seed, 4).reshape(count, 8)
    jobs = []
    t = 0.0
    for j in range(count):
        if rate_per_s > 0:
            t += -math.log1p(-u[j, 0]) / rate_per_s
        n = int(math.floor(math.exp(math.log(1e3) + u[j, 1] * (math.log(n_max) - math.log(1e3)))))
        k = int(round(math.exp(u[j, 2] * math.log(500.0))))
        if j % 2 == 0:
            b = int(round(math.exp(u[j, 3] * math.log(64.0))))
            jobs.append(Job(j, t, max(k, 1), "banded", n, band=b))
        else:
            mean = math.exp(math.log(8.0) + u[j, 4] * (math.log(64.0) - math.log(8.0)))
            s = 0.1 + 1.1 * u[j, 5]
            jobs.append(Job(j, t, max(k, 1), "random", n, mean=mean, s=s))
    return jobs
