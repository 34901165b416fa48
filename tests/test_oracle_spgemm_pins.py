"""Pins of the oracle's numeric product (the consumer of the prediction).

The numeric product is C = A.B by definition; these tests tie the oracle to
things computed independently of its code: dense matrix products, scipy's
sparse product, identities (A.I = A, I.B = B), the closed form of the squared
27-point stencil, the precise structure and row FLOP of the structure oracle,
and a brute-force statement of the predicted-capacity slot layout.
"""
import math

import numpy as np
import pytest

import workloads
from tests.csr_util import from_rows, random_csr


def _dense(M, vals):
    D = np.zeros((M.nrows, M.ncols))
    for i in range(M.nrows):
        for e in range(M.rpt[i], M.rpt[i + 1]):
            D[i, M.col[e]] += vals[e]
    return D


def _pattern_product(A, B):
    PA = np.zeros((A.nrows, A.ncols), dtype=np.int64)
    PB = np.zeros((B.nrows, B.ncols), dtype=np.int64)
    for i in range(A.nrows):
        for e in range(A.rpt[i], A.rpt[i + 1]):
            PA[i, A.col[e]] += 1
    for i in range(B.nrows):
        for e in range(B.rpt[i], B.rpt[i + 1]):
            PB[i, B.col[e]] += 1
    return PA @ PB  # (i, j): number of intermediate products


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_spgemm_matches_dense_product(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    # unsorted rows with duplicate entries: duplicates add
    A = random_csr(rng, 37, 23, 0.2, dup_prob=0.3)
    B = random_csr(rng, 23, 41, 0.15, dup_prob=0.3)
    av = workloads.values(A.nnz, seed, "int")
    bv = workloads.values(B.nnz, seed + 7, "int")
    rpt, col, val, aab, terms = oracle_mod.spgemm(A, av, B, bv)
    P = _pattern_product(A, B)
    D = _dense(A, av) @ _dense(B, bv)
    for i in range(A.nrows):
        cols = col[rpt[i]:rpt[i + 1]]
        assert list(cols) == sorted(set(np.nonzero(P[i])[0])), i  # structure, increasing
        assert np.array_equal(val[rpt[i]:rpt[i + 1]], D[i, cols])  # integer values: exact
        assert np.array_equal(terms[rpt[i]:rpt[i + 1]], P[i, cols])
    # sum of |a b| over the terms of an entry
    DA = np.abs(_dense(A, np.abs(av))) @ np.abs(_dense(B, np.abs(bv)))
    for i in range(A.nrows):
        cols = col[rpt[i]:rpt[i + 1]]
        assert np.array_equal(aab[rpt[i]:rpt[i + 1]], DA[i, cols])


def test_spgemm_matches_scipy(oracle_mod):
    sp = pytest.importorskip("scipy.sparse")
    A = workloads.uniform(500, 300, 6, 3)
    B = workloads.uniform(300, 700, 5, 4)
    av = workloads.values(A.nnz, 5)
    bv = workloads.values(B.nnz, 6)
    rpt, col, val, _, _ = oracle_mod.spgemm(A, av, B, bv)
    SA = sp.csr_matrix((av, A.col, A.rpt.astype(np.int64)), shape=(A.nrows, A.ncols))
    SB = sp.csr_matrix((bv, B.col, B.rpt.astype(np.int64)), shape=(B.nrows, B.ncols))
    C = (SA @ SB).tocsr()
    C.sort_indices()
    # (random real values: no sum cancels to exactly zero, so scipy keeps every entry)
    assert np.array_equal(C.indptr, rpt)
    assert np.array_equal(C.indices, col)
    np.testing.assert_allclose(val, C.data, rtol=1e-12, atol=1e-14)


def test_spgemm_identity(oracle_mod):
    A = workloads.rmat(1 << 10, 8, 2)
    av = workloads.values(A.nnz, 9)
    n = A.ncols
    I = from_rows([[i] for i in range(n)], n)
    ones = np.ones(n)
    rpt, col, val, _, terms = oracle_mod.spgemm(A, av, I, ones)
    assert np.array_equal(rpt, A.rpt.astype(np.int64))
    for i in range(A.nrows):
        order = np.argsort(A.col[A.rpt[i]:A.rpt[i + 1]], kind="stable")
        assert np.array_equal(col[rpt[i]:rpt[i + 1]], A.col[A.rpt[i]:A.rpt[i + 1]][order])
        assert np.array_equal(val[rpt[i]:rpt[i + 1]], av[A.rpt[i]:A.rpt[i + 1]][order])
    assert np.all(terms == 1)
    # I.A = A as well
    rpt2, col2, val2, _, _ = oracle_mod.spgemm(I, ones, A, av)
    assert np.array_equal(rpt2, rpt) and np.array_equal(col2, col) and np.array_equal(val2, val)


def test_spgemm_stencil_closed_form(oracle_mod):
    # all-ones 27-point stencil S = T (x) T (x) T with T tridiagonal ones, so
    # S^2 = T^2 (x) T^2 (x) T^2 and T^2[x][y] = #{z in [0,n) : |x-z| <= 1, |z-y| <= 1}
    n = 6
    S = workloads.stencil27(n)
    ones = np.ones(S.nnz)
    rpt, col, val, _, _ = oracle_mod.spgemm(S, ones, S, ones)

    def t2(x, y):
        return sum(1 for z in range(n) if abs(x - z) <= 1 and abs(z - y) <= 1)

    for p in range(S.nrows):
        px, py, pz = p // (n * n), (p // n) % n, p % n
        want = {}
        for qx in range(max(0, px - 2), min(n, px + 3)):
            for qy in range(max(0, py - 2), min(n, py + 3)):
                for qz in range(max(0, pz - 2), min(n, pz + 3)):
                    v = t2(px, qx) * t2(py, qy) * t2(pz, qz)
                    if v:
                        want[(qx * n + qy) * n + qz] = float(v)
        got = dict(zip(col[rpt[p]:rpt[p + 1]].tolist(), val[rpt[p]:rpt[p + 1]].tolist()))
        assert got == want, p


def test_spgemm_structure_agrees_with_precise_method(oracle_mod):
    A = workloads.zipf(2000, 6, 7)
    av = workloads.values(A.nnz, 1)
    rpt, col, val, _, terms = oracle_mod.spgemm(A, av, A, av)
    counts, st = oracle_mod.exact(A, A)
    assert np.array_equal(np.diff(rpt), counts)
    rf, F = oracle_mod.row_flop(A, A)
    assert int(terms.sum()) == F
    per_row = np.add.reduceat(terms.astype(np.int64), rpt[:-1]) if rpt[-1] else np.zeros(0)
    nz = np.diff(rpt) > 0
    assert np.array_equal(per_row[nz], np.asarray(rf)[nz])


def test_spgemm_empty_inputs(oracle_mod):
    A = from_rows([[], [], []], 4)
    B = from_rows([[0, 1], [], [2], [3]], 5)
    rpt, col, val, _, _ = oracle_mod.spgemm(A, np.zeros(0), B, np.ones(B.nnz))
    assert list(rpt) == [0, 0, 0, 0] and col.size == 0
    A2 = from_rows([[1], [1, 1]], 4)  # names only an empty B row (twice)
    rpt, col, _, _, _ = oracle_mod.spgemm(A2, np.ones(3), B, np.ones(B.nnz))
    assert list(rpt) == [0, 0, 0] and col.size == 0


def test_spgemm_layout_brute_force(oracle_mod):
    rng = np.random.default_rng(5)
    N = 50
    for margin in (0, 1, 10, 33, 100, 250):
        cap = rng.integers(-5, 70, 400)
        counts = rng.integers(0, N + 1, 400)
        nnz = slots = orows = onnz = 0
        for c, k in zip(cap.tolist(), counts.tolist()):
            c = min(max(c, 0), N)
            s = min(N, c + math.ceil(c * margin / 100))
            nnz += k
            slots += s
            if k > s:
                orows += 1
                onnz += k
        got = oracle_mod.spgemm_layout(cap, margin, counts, N)
        assert got == {"nnz": nnz, "slot_entries": slots, "overflow_rows": orows,
                       "overflow_nnz": onnz}


def test_spgemm_layout_special_cases(oracle_mod):
    A = workloads.uniform(3000, 3000, 7, 2)
    counts, _ = oracle_mod.exact(A, A)
    rf, F = oracle_mod.row_flop(A, A)
    Z = int(counts.sum())
    # the precise structure as capacity: nothing overflows, slots = NNZ(C)
    assert oracle_mod.spgemm_layout(counts, 0, counts, A.ncols) == {
        "nnz": Z, "slot_entries": Z, "overflow_rows": 0, "overflow_nnz": 0}
    # the upper bound (row FLOP) as capacity: nothing overflows, slots = F (rf <= N here)
    lay = oracle_mod.spgemm_layout(rf, 0, counts, A.ncols)
    assert lay["slot_entries"] == F and lay["overflow_rows"] == 0
    # no capacity: every non-empty row overflows
    lay = oracle_mod.spgemm_layout(np.zeros(A.nrows, dtype=np.int64), 50, counts, A.ncols)
    assert lay["overflow_rows"] == int((counts > 0).sum()) and lay["overflow_nnz"] == Z
