"""Seeded synthetic CSR workloads (int32 indices; seeded values for the numeric product).

The paper evaluates on 25 SuiteSparse matrices and their pairwise products
(Sec. VI, Table II).  Those files are not shipped here; these generators stand
in for them with the shapes named by the benchmark configurations:

* ``uniform``   -- exactly ``d`` distinct uniform columns per row;
* ``rmat``      -- plain R-MAT (a, b, c, d) = (0.57, 0.19, 0.19, 0.05), edges
                   ``avg_deg * 2**scale``, duplicates merged (power-law rows);
* ``banded``    -- ``d`` distinct uniform columns within half-width ``hw``;
* ``blockdiag`` -- ``d`` distinct uniform columns inside 256-wide diagonal blocks;
* ``zipf``      -- Zipf(1.5) row lengths scaled to mean ``d``, uniform columns;
* ``stencil27`` -- the 27-point stencil on an n^3 grid, natural ordering.

This module holds no part of the prediction method; the oracle and the GPU
path both read its matrices.  The C generator (``wl_gen.c``) is built into
``libworkloads.so`` next to this file.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wl_gen.c")
_LIB = os.path.join(_HERE, "libworkloads.so")

UNIFORM, BANDED, BLOCKDIAG, ZIPF = 1, 2, 3, 4
STRUCTURES = ("uniform", "rmat", "banded", "blockdiag", "zipf")


def build(force: bool = False) -> str:
    """Compile the generator library with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, u64, i32p = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
        lib.wl_rowgen_rowlen.argtypes = [ctypes.c_int, i64, i64, i64, i64, u64, i32p,
                                         ctypes.POINTER(ctypes.c_double)]
        lib.wl_rowgen_fill.argtypes = [ctypes.c_int, i64, i64, i64, i64, u64, i32p, i32p]
        lib.wl_stencil27_rowlen.argtypes = [i64, i32p]
        lib.wl_stencil27_fill.argtypes = [i64, i32p, i32p]
        lib.wl_rmat.argtypes = [ctypes.c_int, i64, i64, i64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, u64, ctypes.POINTER(ctypes.c_void_p),
                                ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(i64)]
        lib.wl_free.argtypes = [ctypes.c_void_p]
        for f in (lib.wl_rowgen_rowlen, lib.wl_rowgen_fill, lib.wl_stencil27_rowlen,
                  lib.wl_stencil27_fill, lib.wl_rmat):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class CSR:
    """Structure-only CSR: rpt int32[nrows+1], col int32[nnz]."""
    nrows: int
    ncols: int
    rpt: np.ndarray
    col: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.rpt.astype(np.int64))


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _rpt_from_lengths(lengths: np.ndarray) -> np.ndarray:
    rpt = np.zeros(lengths.shape[0] + 1, dtype=np.int64)
    np.cumsum(lengths, out=rpt[1:])
    return rpt


def _finish(nrows, ncols, rpt64, col, name) -> CSR:
    if rpt64[-1] > np.iinfo(np.int32).max:
        raise ValueError(f"{name}: nnz {rpt64[-1]} does not fit int32 row pointers")
    return CSR(nrows, ncols, rpt64.astype(np.int32), col, name)


def _rowgen(kind: int, nrows: int, ncols: int, d: int, param: int, seed: int, name: str) -> CSR:
    lib = _load()
    lens = np.empty(nrows, dtype=np.int32)
    mean = ctypes.c_double(0.0)
    rc = lib.wl_rowgen_rowlen(kind, nrows, ncols, d, param, seed, _ptr(lens), ctypes.byref(mean))
    if rc:
        raise ValueError(f"{name}: generator rejected its parameters ({rc})")
    rpt = _rpt_from_lengths(lens)
    col = np.empty(int(rpt[-1]), dtype=np.int32)
    rc = lib.wl_rowgen_fill(kind, nrows, ncols, d, param, seed, _ptr(rpt), _ptr(col))
    if rc:
        raise ValueError(f"{name}: generator failed ({rc})")
    return _finish(nrows, ncols, rpt, col, name)


def uniform(nrows: int, ncols: int, d: int, seed: int) -> CSR:
    return _rowgen(UNIFORM, nrows, ncols, d, 0, seed, f"uniform{nrows}x{ncols}d{d}s{seed}")


def banded(n: int, d: int, seed: int, hw: int = 64) -> CSR:
    return _rowgen(BANDED, n, n, d, hw, seed, f"banded{n}d{d}hw{hw}s{seed}")


def blockdiag(n: int, d: int, seed: int, block: int = 256) -> CSR:
    return _rowgen(BLOCKDIAG, n, n, d, block, seed, f"blockdiag{n}d{d}b{block}s{seed}")


def zipf(n: int, d: int, seed: int, s: float = 1.5) -> CSR:
    return _rowgen(ZIPF, n, n, d, int(round(s * 1000)), seed, f"zipf{n}d{d}s{seed}")


def stencil27(n: int) -> CSR:
    lib = _load()
    m = n * n * n
    lens = np.empty(m, dtype=np.int32)
    lib.wl_stencil27_rowlen(n, _ptr(lens))
    rpt = _rpt_from_lengths(lens)
    col = np.empty(int(rpt[-1]), dtype=np.int32)
    lib.wl_stencil27_fill(n, _ptr(rpt), _ptr(col))
    return _finish(m, m, rpt, col, f"stencil27_{n}")


def rmat(n: int, avg_deg: float, seed: int, a: float = 0.57, b: float = 0.19,
         c: float = 0.19) -> CSR:
    """Square R-MAT with n rows (2^ceil(log2 n) recursion), avg_deg*n edges, merged."""
    lib = _load()
    scale = max(0, int(math.ceil(math.log2(n)))) if n > 1 else 0
    nedges = int(round(avg_deg * n))
    rp, cp, nnz = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_int64()
    rc = lib.wl_rmat(scale, n, n, nedges, a, b, c, seed, ctypes.byref(rp), ctypes.byref(cp),
                     ctypes.byref(nnz))
    if rc:
        raise ValueError(f"rmat: generator failed ({rc})")
    try:
        rpt = np.ctypeslib.as_array(ctypes.cast(rp, ctypes.POINTER(ctypes.c_int64)),
                                    shape=(n + 1,)).copy()
        col = (np.ctypeslib.as_array(ctypes.cast(cp, ctypes.POINTER(ctypes.c_int32)),
                                     shape=(max(nnz.value, 1),))[: nnz.value].copy())
    finally:
        lib.wl_free(rp)
        lib.wl_free(cp)
    return _finish(n, n, rpt, col, f"rmat{n}d{avg_deg}s{seed}")


def make(structure: str, n: int, d: int, seed: int) -> CSR:
    """One square matrix of the batched sweep's five structure families."""
    if structure == "uniform":
        return uniform(n, n, d, seed)
    if structure == "rmat":
        return rmat(n, d, seed)
    if structure == "banded":
        return banded(n, d, seed, 64)
    if structure == "blockdiag":
        return blockdiag(n, d, seed, 256)
    if structure == "zipf":
        return zipf(n, d, seed, 1.5)
    raise ValueError(f"unknown structure {structure!r}")


# ------------------------------------------------------------------- values

def values(n: int, seed: int, kind: str = "uniform") -> np.ndarray:
    """Seeded float64 values for the ``n`` stored entries of a matrix.

    ``uniform``: independent draws from U[-1, 1).  ``int``: small integers in
    [-4, 4] without 0, so products and their sums are exact in float64 and
    every summation order gives the same result."""
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.uniform(-1.0, 1.0, n)
    if kind == "int":
        v = rng.integers(1, 5, n).astype(np.float64)
        return np.where(rng.integers(0, 2, n) == 1, v, -v)
    if kind == "ones":
        return np.ones(n, dtype=np.float64)
    raise ValueError(f"unknown value kind {kind!r}")


# ---------------------------------------------------------------- workloads

@dataclass
class Workload:
    """One product C = A.B to predict: inputs, sample rate and sampler seed."""
    name: str
    A: CSR
    B: CSR
    rate: float
    seed: int

    @property
    def aliased(self) -> bool:
        return self.A is self.B


def uniform4096(gen_seed: int = 1) -> Workload:
    """C = A.A, A 4096x4096 with 8 distinct uniform columns per row, 1% sampling."""
    A = uniform(4096, 4096, 8, gen_seed)
    return Workload("uniform4096_d8", A, A, 0.01, 1000 + gen_seed)


def rmat20(gen_seed: int = 1) -> Workload:
    """C = A.A, A 2^20 x 2^20 R-MAT (0.57,0.19,0.19,0.05), 16 edges/row merged, 0.5%."""
    A = rmat(1 << 20, 16, gen_seed)
    return Workload("rmat20_d16", A, A, 0.005, 1000 + gen_seed)


def stencil128(gen_seed: int = 1) -> Workload:
    """C = A.A, A the 27-point stencil on a 128^3 grid, 0.5% sampling."""
    A = stencil27(128)
    return Workload("stencil27_128", A, A, 0.005, 1000 + gen_seed)


def stencil128_x_uniform(gen_seed: int = 1) -> Workload:
    """C = A.B, A the 128^3 27-point stencil, B 2,097,152 x 65,536 with 4 uniform cols/row."""
    A = stencil27(128)
    B = uniform(A.ncols, 65536, 4, gen_seed)
    return Workload("stencil27_128_x_uniform65536_d4", A, B, 0.005, 1000 + gen_seed)


SWEEP_SIZES = (1 << 12, 1 << 14, 1 << 16, 1 << 18, 1 << 20)
SWEEP_DEGREES = (2, 4, 8, 16, 32)
SWEEP_SEEDS = (1, 2, 3, 4, 5)


def sweep_cases(sizes=SWEEP_SIZES, degrees=SWEEP_DEGREES, structures=STRUCTURES,
                seeds=SWEEP_SEEDS):
    """Parameters (structure, n, d, gen_seed, rate, sampler_seed) of the 625-case sweep."""
    out = []
    for n in sizes:
        for d in degrees:
            for s in structures:
                for g in seeds:
                    out.append((s, n, d, g, 0.01, 1000 + g))
    return out


def sweep_workload(case) -> Workload:
    s, n, d, g, rate, seed = case
    A = make(s, n, d, g)
    return Workload(f"{s}_n{n}_d{d}_s{g}", A, A, rate, seed)


def num_threads() -> int:
    return int(_load().wl_num_threads())
