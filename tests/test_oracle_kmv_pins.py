"""Pins of the oracle's sketch estimator (Sec. III: Amossen's k minimum values
with BHash's row and column sampling).

Tied to: the precise structure and row FLOP of the structure oracle (all rows
and columns kept), the pinned splitmix64 row sampler (which rows and columns
are kept), a dense brute force of the sampled product's pairs hashed with the
pinned splitmix64 stream, and the sketch's known accuracy (relative standard
error about 1/sqrt(k)).
"""
import math

import numpy as np
import pytest

import workloads
from tests.csr_util import random_csr


def _count_dense(M):
    D = np.zeros((M.nrows, M.ncols), dtype=np.int64)
    for i in range(M.nrows):
        for e in range(M.rpt[i], M.rpt[i + 1]):
            D[i, M.col[e]] += 1
    return D


def test_kmv_all_kept_is_exact(oracle_mod):
    A = workloads.zipf(3000, 6, 3)
    counts, st = oracle_mod.exact(A, A)
    _, F = oracle_mod.row_flop(A, A)
    r = oracle_mod.kmv(A, A, 1.0, 10 ** 9, 7)  # k above NNZ(C): the sketch holds every value
    assert r["rows_kept"] == A.nrows and r["cols_kept"] == A.ncols
    assert r["products"] == F
    assert r["distinct"] == st.out_sum  # (no two pairs share a 53-bit hash here)
    assert r["kth_hash"] == 0 and r["nnz_estimate"] == float(st.out_sum)


@pytest.mark.parametrize("rate", [0.05, 0.3])
def test_kmv_kept_rows_and_columns_follow_the_sampler(oracle_mod, rate):
    A = workloads.uniform(5000, 7000, 4, 2)
    B = workloads.uniform(7000, 6000, 3, 3)
    seed = 12345
    r = oracle_mod.kmv(A, B, rate, 64, seed)
    assert r["rows_kept"] == len(oracle_mod.sample_rows(A.nrows, rate, seed))
    assert r["cols_kept"] == len(oracle_mod.sample_rows(B.ncols, rate, seed + 1))
    for n, kept in ((A.nrows, r["rows_kept"]), (B.ncols, r["cols_kept"])):
        sd = math.sqrt(n * rate * (1 - rate))
        assert abs(kept - n * rate) < 5 * sd


@pytest.mark.parametrize("seed,rate,k", [(1, 1.0, 20), (2, 0.5, 7), (3, 0.35, 3), (4, 0.5, 400)])
def test_kmv_brute_force(oracle_mod, seed, rate, k):
    rng = np.random.default_rng(seed)
    A = random_csr(rng, 60, 40, 0.15, dup_prob=0.3)
    B = random_csr(rng, 40, 50, 0.2, dup_prob=0.3)
    P = _count_dense(A) @ _count_dense(B)
    T = oracle_mod.rate_threshold(rate)
    rows = [i for i in range(A.nrows) if (oracle_mod.splitmix64(seed, i) >> 11) < T]
    cols = [j for j in range(B.ncols) if (oracle_mod.splitmix64(seed + 1, j) >> 11) < T]
    prods = int(P[np.ix_(rows, cols)].sum()) if rows and cols else 0
    hv = sorted({oracle_mod.splitmix64(seed + 2, i * B.ncols + j) >> 11
                 for i in rows for j in cols if P[i, j] > 0})
    r = oracle_mod.kmv(A, B, rate, k, seed)
    assert r["rows_kept"] == len(rows) and r["cols_kept"] == len(cols)
    assert r["products"] == prods
    assert r["distinct"] == len(hv)
    assert r["kth_hash"] == (hv[k - 1] if len(hv) >= k else 0)
    if len(hv) >= k:
        assert r["nnz_sample"] == k / (hv[k - 1] / 2.0 ** 53)
    else:
        assert r["nnz_sample"] == float(len(hv))


def test_kmv_accuracy_all_kept(oracle_mod):
    # relative standard error of k / v is about 1/sqrt(k): over 8 seeds the
    # mean estimate is within 5 standard errors of the mean
    A = workloads.stencil27(16)
    _, st = oracle_mod.exact(A, A)
    Z, k = st.out_sum, 256
    est = [oracle_mod.kmv(A, A, 1.0, k, s)["nnz_estimate"] for s in range(8)]
    assert all(abs(e / Z - 1) < 6 / math.sqrt(k) for e in est)
    assert abs(np.mean(est) / Z - 1) < 5 / math.sqrt(8 * k)


def test_kmv_sampled_estimate_scales(oracle_mod):
    # with p = 1/10 on both sides the estimate divides the sample's NNZ by p_r p_c
    A = workloads.uniform(20000, 20000, 8, 5)
    r = oracle_mod.kmv(A, A, 0.1, 128, 9)
    pr, pc = r["rows_kept"] / A.nrows, r["cols_kept"] / A.ncols
    assert r["nnz_estimate"] == r["nnz_sample"] / (pr * pc)
    _, st = oracle_mod.exact(A, A)
    assert abs(r["nnz_estimate"] / st.out_sum - 1) < 0.5


def test_kmv_nothing_kept(oracle_mod):
    A = workloads.uniform(100, 100, 4, 1)
    r = oracle_mod.kmv(A, A, 0.0, 16, 1)
    assert r["rows_kept"] == 0 and r["products"] == 0 and r["distinct"] == 0
    assert r["nnz_sample"] == 0.0 and r["nnz_estimate"] is None
