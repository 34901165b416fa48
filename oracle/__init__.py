"""Serial CPU oracle for sampled-compression-ratio structure prediction.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's CPU
baseline are the only callers.  The oracle shares no code with the GPU
library; both read the same seeded matrices from ``workloads``.

The arithmetic lives in ``ssp_oracle.c`` (plain serial C, built with gcc into
``liboracle.so`` next to this file).  This module marshals numpy arrays and
adds the accuracy statistics of Sec. VI-A, computed in exact rationals.

Paper anchors (Du et al., arXiv 2207.13848):
  * row FLOP and F ................ Sec. V-A, Alg. 1; Eq. (1)
  * row sampling of A ............. Sec. IV-A; Alg. 2 and Sec. V-B (paper mode)
  * exact NNZ of sampled rows ..... Sec. IV-B; Alg. 2
  * proposed estimate Z2*, rows ... Sec. IV-D, Eq. (4); Alg. 2
  * reference design Z1* .......... Sec. IV-C, Eq. (2)
  * symmetric F* and eps_f ........ Eq. (3)
  * error identity ................ Eq. (5)
  * precise method (exact) ........ Sec. I (symbolic phase)
  * numeric product (consumer) .... Sec. I (the output the prediction sizes):
                                    the definition of C = A.B, and the slot
                                    layout of a predicted-capacity allocation
  * the sketch estimator (KMV) .... Sec. III (Amossen et al.; BHash's p = 1/10
                                    row and column sampling, NNZ(C')/p^2)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ssp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# the mutation tests load deliberately broken copies through this override
_LIB = os.environ.get("SSP_ORACLE_LIB_OVERRIDE", _LIB)

FLAG_EMPTY_SAMPLE = 1
BERNOULLI, PAPER = 0, 1


def build(force: bool = False) -> str:
    if "SSP_ORACLE_LIB_OVERRIDE" in os.environ:
        return _LIB
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in
                ("total_flop", "n_sampled", "sample_flop", "sample_nnz", "out_sum", "nrows",
                 "flags", "a_sample_nnz")]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        vp, i64, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64
        lib.orc_check_csr.argtypes = [i64, i64, i64, vp, vp]
        lib.orc_check_csr.restype = ctypes.c_int
        lib.orc_row_flop.argtypes = [i64, vp, vp, vp, vp, ctypes.POINTER(u64)]
        lib.orc_row_flop.restype = None
        lib.orc_splitmix64.argtypes = [u64, u64]
        lib.orc_splitmix64.restype = u64
        lib.orc_rate_threshold.argtypes = [ctypes.c_double]
        lib.orc_rate_threshold.restype = u64
        lib.orc_sample_bernoulli.argtypes = [i64, u64, u64, vp]
        lib.orc_sample_bernoulli.restype = i64
        lib.orc_sample_paper.argtypes = [i64, u64, vp]
        lib.orc_sample_paper.restype = i64
        lib.orc_paper_sample_num.argtypes = [i64]
        lib.orc_paper_sample_num.restype = i64
        lib.orc_ceil_mul_div_wide.argtypes = [u64, u64, u64, u64, u64]
        lib.orc_ceil_mul_div_wide.restype = u64
        for name in ("orc_predict", "orc_reference"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int
        lib.orc_predict.argtypes = [i64, i64, vp, vp, vp, vp, ctypes.c_double, u64, ctypes.c_int,
                                    vp, vp, ctypes.POINTER(_Stats)]
        lib.orc_reference.argtypes = [i64, i64, vp, vp, vp, vp, ctypes.c_double, u64,
                                      ctypes.c_int, vp, ctypes.POINTER(_Stats)]
        lib.orc_exact.argtypes = [i64, i64, vp, vp, vp, vp, vp, ctypes.POINTER(_Stats)]
        lib.orc_exact.restype = ctypes.c_int
        lib.orc_rows_nnz.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp]
        lib.orc_rows_nnz.restype = ctypes.c_int
        lib.orc_spgemm.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.orc_spgemm.restype = ctypes.c_int
        lib.orc_kmv.argtypes = [i64, i64, vp, vp, vp, vp, u64, u64, u64] + [ctypes.POINTER(u64)] * 5
        lib.orc_kmv.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


@dataclass
class Stats:
    total_flop: int   # F
    n_sampled: int    # n_s
    sample_flop: int  # f*
    sample_nnz: int   # z*
    out_sum: int      # sum of the per-row outputs
    nrows: int        # M
    flags: int
    a_sample_nnz: int  # stored entries of A in the sampled rows

    @classmethod
    def _from(cls, s: _Stats) -> "Stats":
        return cls(s.total_flop, s.n_sampled, s.sample_flop, s.sample_nnz, s.out_sum, s.nrows,
                   s.flags, s.a_sample_nnz)

    # --- Eq. (2)-(4) as exact rationals (None where undefined) --------------
    @property
    def z2_star(self):
        """Proposed estimate Z2* = F z*/f* (Eq. (4))."""
        if self.sample_flop == 0:
            return None
        return Fraction(self.total_flop * self.sample_nnz, self.sample_flop)

    @property
    def z1_star(self):
        """Reference estimate Z1* = z*/p, p = n_s/M (Eq. (2))."""
        if self.n_sampled == 0:
            return None
        return Fraction(self.sample_nnz * self.nrows, self.n_sampled)

    @property
    def f_star(self):
        """Symmetric FLOP estimate F* = f*/p (Eq. (3))."""
        if self.n_sampled == 0:
            return None
        return Fraction(self.sample_flop * self.nrows, self.n_sampled)


def _csr_args(A, B):
    if A.ncols != B.nrows:
        raise ValueError("A.ncols != B.nrows")
    return (A.nrows, A.ncols, _i32(A.rpt), _i32(A.col), _i32(B.rpt), _i32(B.col))


def check_csr(M) -> int:
    rpt, col = _i32(M.rpt), _i32(M.col)
    return int(_load().orc_check_csr(M.nrows, M.ncols, col.shape[0], _p(rpt), _p(col)))


def row_flop(A, B):
    """(row_flop uint64[M], F) by Alg. 1."""
    M, K, ar, ac, br, bc = _csr_args(A, B)
    out = np.zeros(M, dtype=np.uint64)
    tot = ctypes.c_uint64()
    _load().orc_row_flop(M, _p(ar), _p(ac), _p(br), _p(out), ctypes.byref(tot))
    return out, int(tot.value)


def splitmix64(seed: int, i: int) -> int:
    return int(_load().orc_splitmix64(seed & (2**64 - 1), i))


def rate_threshold(rate: float) -> int:
    return int(_load().orc_rate_threshold(rate))


def sample_rows(M: int, rate: float, seed: int, mode: int = BERNOULLI) -> np.ndarray:
    lib = _load()
    if mode == PAPER:
        out = np.empty(max(lib.orc_paper_sample_num(M), 1), dtype=np.int32)
        n = lib.orc_sample_paper(M, seed, _p(out))
    else:
        out = np.empty(max(M, 1), dtype=np.int32)
        n = lib.orc_sample_bernoulli(M, seed, lib.orc_rate_threshold(rate), _p(out))
    return out[:n].copy()


def ceil_mul_div_wide(a: int, q: int, d: int) -> int:
    """ceil(a q / d) as the reference design computes it (64-bit a, 128-bit
    q and d, a quotient below 2^64)."""
    m = (1 << 64) - 1
    return int(_load().orc_ceil_mul_div_wide(a, q >> 64, q & m, d >> 64, d & m))


def paper_sample_num(M: int) -> int:
    return int(_load().orc_paper_sample_num(M))


def predict(A, B, rate: float, seed: int, mode: int = BERNOULLI):
    """(nnz_pred int64[M], row_flop uint64[M], Stats) of the proposed method."""
    M, K, ar, ac, br, bc = _csr_args(A, B)
    pred = np.zeros(max(M, 1), dtype=np.int64)
    rf = np.zeros(max(M, 1), dtype=np.uint64)
    st = _Stats()
    rc = _load().orc_predict(M, K, _p(ar), _p(ac), _p(br), _p(bc), rate, seed & (2**64 - 1),
                             mode, _p(pred), _p(rf), ctypes.byref(st))
    if rc:
        raise ValueError(f"oracle predict failed ({rc})")
    return pred[:M], rf[:M], Stats._from(st)


def reference(A, B, rate: float, seed: int, mode: int = BERNOULLI):
    """(nnz_ref int64[M], Stats) of the reference design."""
    M, K, ar, ac, br, bc = _csr_args(A, B)
    out = np.zeros(max(M, 1), dtype=np.int64)
    st = _Stats()
    rc = _load().orc_reference(M, K, _p(ar), _p(ac), _p(br), _p(bc), rate, seed & (2**64 - 1),
                               mode, _p(out), ctypes.byref(st))
    if rc:
        raise ValueError(f"oracle reference failed ({rc})")
    return out[:M], Stats._from(st)


def exact(A, B):
    """(nnz_exact int64[M], Stats with out_sum = Z) of the precise method."""
    M, K, ar, ac, br, bc = _csr_args(A, B)
    out = np.zeros(max(M, 1), dtype=np.int64)
    st = _Stats()
    rc = _load().orc_exact(M, K, _p(ar), _p(ac), _p(br), _p(bc), _p(out), ctypes.byref(st))
    if rc:
        raise ValueError(f"oracle exact failed ({rc})")
    return out[:M], Stats._from(st)


def rows_nnz(A, B, rows):
    """Exact nnz and row FLOP of the listed rows only."""
    M, K, ar, ac, br, bc = _csr_args(A, B)
    rows = _i32(rows)
    nnz = np.zeros(max(rows.shape[0], 1), dtype=np.int64)
    rf = np.zeros(max(rows.shape[0], 1), dtype=np.uint64)
    rc = _load().orc_rows_nnz(rows.shape[0], _p(rows), _p(ar), _p(ac), _p(br), _p(bc), _p(nnz),
                              _p(rf))
    if rc:
        raise ValueError(f"oracle rows_nnz failed ({rc})")
    return nnz[: rows.shape[0]], rf[: rows.shape[0]]


# ------------------------------------------- the consumer (numeric product)

def spgemm(A, A_val, B, B_val):
    """C = A.B with values, by the definition (``orc_spgemm``).

    Returns ``(C_rpt int64[M+1], C_col int32, C_val f64, C_abs f64,
    C_terms int32)``: rows with increasing columns; ``C_abs`` is the sum of
    |a*b| over an entry's terms and ``C_terms`` their number, which bound the
    rounding error of any order of summation."""
    M, K, ar, ac, br, bc = _csr_args(A, B)
    av = np.ascontiguousarray(A_val, dtype=np.float64)
    bv = np.ascontiguousarray(B_val, dtype=np.float64)
    if av.shape[0] != ac.shape[0] or bv.shape[0] != bc.shape[0]:
        raise ValueError("value arrays must match the column arrays")
    counts, _ = exact(A, B)
    rpt = np.zeros(M + 1, dtype=np.int64)
    np.cumsum(counts, out=rpt[1:])
    Z = int(rpt[M])
    col = np.zeros(max(Z, 1), dtype=np.int32)
    val = np.zeros(max(Z, 1), dtype=np.float64)
    aab = np.zeros(max(Z, 1), dtype=np.float64)
    terms = np.zeros(max(Z, 1), dtype=np.int32)
    N = int(B.ncols)
    av1 = av if av.size else np.zeros(1)  # (kept alive across the call)
    bv1 = bv if bv.size else np.zeros(1)
    rc = _load().orc_spgemm(M, N, _p(ar), _p(ac), _p(av1), _p(br), _p(bc), _p(bv1), _p(rpt),
                            _p(col), _p(val), _p(aab), _p(terms))
    if rc:
        raise ValueError(f"oracle spgemm failed ({rc})")
    return rpt, col[:Z], val[:Z], aab[:Z], terms[:Z]


def spgemm_layout(row_cap, margin_pct: int, counts, ncols: int) -> dict:
    """Integer outcome of the predicted-capacity consumer.

    Row i gets a slot of ``min(N, c + ceil(c * margin_pct / 100))`` entries,
    ``c = row_cap[i]`` clamped to [0, N] (a row of C has at most N entries).
    A row whose nonzero count exceeds its slot overflows and is recomputed by
    the fallback pass.  Returns nnz, slot_entries, overflow_rows and
    overflow_nnz as Python ints."""
    N = int(ncols)
    cap = np.clip(np.asarray(row_cap, dtype=np.int64), 0, N)
    slot = np.minimum(N, cap + (cap * int(margin_pct) + 99) // 100)
    cnt = np.asarray(counts, dtype=np.int64)
    over = cnt > slot
    return {"nnz": int(cnt.sum()), "slot_entries": int(slot.sum()),
            "overflow_rows": int(over.sum()), "overflow_nnz": int(cnt[over].sum())}


# ------------------------------------------ Sec. III: the sketch estimator

def kmv(A, B, rate: float, k: int, seed: int) -> dict:
    """Amossen's k-minimum-values estimate with BHash's row and column
    sampling (``orc_kmv``; definitions in its comment).  Returns the integer
    results and the estimates: ``nnz_sample`` = k / v (v = the k-th smallest
    distinct hash / 2^53) or the distinct count when there are fewer than k,
    ``nnz_estimate`` = nnz_sample / (p_r p_c) with the realised proportions
    p_r = rows kept / M and p_c = columns kept / N (None when nothing is kept)."""
    M, K, ar, ac, br, bc = _csr_args(A, B)
    T = rate_threshold(rate)
    out = [ctypes.c_uint64(0) for _ in range(5)]
    rc = _load().orc_kmv(M, int(B.ncols), _p(ar), _p(ac), _p(br), _p(bc), T, seed % (1 << 64),
                         int(k), *[ctypes.byref(o) for o in out])
    if rc:
        raise ValueError(f"oracle kmv failed ({rc})")
    nr, nc, npr, d, kv = (int(o.value) for o in out)
    return dict(rows_kept=nr, cols_kept=nc, products=npr, distinct=d, kth_hash=kv, k=int(k),
                **kmv_estimates(M, int(B.ncols), nr, nc, d, kv, int(k)))


def kmv_estimates(M: int, N: int, nr: int, nc: int, distinct: int, kth: int, k: int) -> dict:
    """The estimates of the sketch from its integer results (float64, the
    order of operations both sides use)."""
    if distinct >= k and kth > 0:
        zs = float(k) / (float(kth) / 9007199254740992.0)
    else:
        zs = float(distinct)
    if nr == 0 or nc == 0:
        return {"nnz_sample": zs, "nnz_estimate": None}
    return {"nnz_sample": zs, "nnz_estimate": zs / ((nr / M) * (nc / N))}


# ------------------------------------------------------- Sec. VI-A accuracy

def compression_ratio(flop: int, nnz: int) -> Fraction:
    """CR = FLOP / NNZ (Table I)."""
    return Fraction(flop, nnz)


def relative_errors(stats: Stats, Z: int) -> dict:
    """eps_1, eps_f, eps_2 of Sec. VI-A as exact rationals, and eps_2 of the
    allocation actually handed out (sum of the per-row ceilings).

    eps_1 = (Z1* - Z)/Z, eps_f = (F* - F)/F, eps_2 = (Z2* - Z)/Z; a quantity
    whose estimate is undefined (empty sample) or whose truth is zero is None.
    """
    out = {"eps1": None, "epsf": None, "eps2": None, "eps2_alloc": None}
    if Z > 0 and stats.z1_star is not None:
        out["eps1"] = stats.z1_star / Z - 1
    if stats.total_flop > 0 and stats.f_star is not None:
        out["epsf"] = stats.f_star / stats.total_flop - 1
    if Z > 0 and stats.z2_star is not None:
        out["eps2"] = stats.z2_star / Z - 1
    if Z > 0:
        out["eps2_alloc"] = Fraction(stats.out_sum, Z) - 1
    return out
