"""Pins of the CPU oracle to things other than itself.

Each test ties one part of the oracle to something fixed independently of its
code: dense brute force, closed forms of special structures, published known
answers of splitmix64, sampling statistics, the paper's printed tables, a
hand-worked example and exact identities of the method (Eq. (4), Eq. (5)).
"""
import csv
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import workloads
from tests.csr_util import from_rows, random_csr, to_count_dense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _csv(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return list(csv.DictReader(line for line in f if not line.startswith("#")))


# ------------------------------------------------------------ sampler (a1)

def test_splitmix64_published_outputs(oracle_mod):
    # first three outputs of splitmix64 with initial state 0 (Vigna's splitmix64.c)
    assert oracle_mod.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert oracle_mod.splitmix64(0, 1) == 0x6E789E6AA1B965F4
    assert oracle_mod.splitmix64(0, 2) == 0x06C45D188009454F


def test_splitmix64_stream_is_keyed_by_seed_and_counter(oracle_mod):
    # output i of the stream seeded with s equals output 0 of the stream seeded
    # with s + i * golden (the state simply advances by the golden increment)
    g = 0x9E3779B97F4A7C15
    for s in (0, 1, 12345, 2**64 - 1):
        for i in (1, 2, 17, 1 << 40):
            assert oracle_mod.splitmix64(s, i) == oracle_mod.splitmix64((s + i * g) % 2**64, 0)


def test_rate_threshold(oracle_mod):
    assert oracle_mod.rate_threshold(0.0) == 0
    assert oracle_mod.rate_threshold(1.0) == 2**53
    assert oracle_mod.rate_threshold(0.5) == 2**52
    assert oracle_mod.rate_threshold(0.01) == math.floor(0.01 * 2**53)
    assert oracle_mod.rate_threshold(float("nan")) == 0


@pytest.mark.parametrize("rate", [0.001, 0.005, 0.01, 0.25])
def test_bernoulli_sample_statistics(oracle_mod, rate):
    M = 1_000_000
    for seed in (1001, 7):
        S = oracle_mod.sample_rows(M, rate, seed)
        assert np.all(np.diff(S) > 0) and (S.size == 0 or (S[0] >= 0 and S[-1] < M))
        mu, sd = M * rate, math.sqrt(M * rate * (1 - rate))
        assert abs(S.size - mu) < 5 * sd
        # uniform over the row range: each half holds about half the sample
        lo = int(np.sum(S < M // 2))
        assert abs(lo - S.size / 2) < 5 * math.sqrt(S.size / 4) + 1


def test_bernoulli_sample_extremes(oracle_mod):
    assert oracle_mod.sample_rows(1000, 0.0, 5).size == 0
    assert np.array_equal(oracle_mod.sample_rows(1000, 1.0, 5), np.arange(1000))
    assert oracle_mod.sample_rows(0, 0.5, 5).size == 0


def test_sample_is_a_pure_function_of_seed_and_row(oracle_mod):
    # membership of row i does not depend on M: a prefix of rows keeps its sample
    S_big = oracle_mod.sample_rows(100_000, 0.05, 3)
    S_small = oracle_mod.sample_rows(50_000, 0.05, 3)
    assert np.array_equal(S_big[S_big < 50_000], S_small)


# -------------------------------------------- paper tables (Sec. VI) pins

def test_table2_compression_ratio_definition(oracle_mod):
    # Table I defines CR = FLOP / NNZ; Table II prints it (2 decimals) for A^2
    for r in _csv("paper_table2.csv"):
        cr = oracle_mod.compression_ratio(int(r["flop_A2"]), int(r["nnz_A2"]))
        assert abs(float(cr) - float(r["cr_A2"])) <= 0.005 + 1e-12, r["name"]
        assert abs(int(r["nnz"]) / int(r["rows"]) - float(r["nnz_per_row"])) <= 0.05 + 1e-12


def test_table3_eq5_identity_holds_on_printed_triples():
    # Eq. (5): eps2 = (eps1 - epsf) / (1 + epsf); the paper states every row of
    # Table III meets it.  Printed values are rounded to 0.01 percentage points,
    # so each carries up to h = 0.005 pp; propagated through Eq. (5) that allows
    # h/(1+epsf) + h(1+eps1)/(1+epsf)^2 from the inputs plus h on eps2 itself.
    h = 0.005 / 100
    for r in _csv("paper_table3.csv"):
        e1, ef, e2 = (float(r[k]) / 100 for k in ("eps1_pct", "epsf_pct", "eps2_pct"))
        tol = h / (1 + ef) + h * (1 + e1) / (1 + ef) ** 2 + h + 1e-12
        assert abs((e1 - ef) / (1 + ef) - e2) <= tol, r["case"]


def test_table3_sample_num_rule(oracle_mod):
    # Sec. V-B: sample_num = min(0.003 M, 300) with M the rows of A; Table III
    # prints 140 for rma10 (M = 46,835, 0.003 M = 140.5) and 300 elsewhere
    rows_of = {r["name"]: int(r["rows"]) for r in _csv("paper_table2.csv")}
    for r in _csv("paper_table3.csv"):
        assert oracle_mod.paper_sample_num(rows_of[r["A"]]) == int(r["sample_num"]), r["case"]


# ----------------------------------------------- brute force (a2, a3, a7)

@pytest.mark.parametrize("seed", range(12))
def test_row_flop_and_exact_vs_dense_brute_force(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    M, K, N = rng.integers(1, 40, size=3)
    dens_a, dens_b = rng.uniform(0.0, 0.6, size=2)
    A = random_csr(rng, int(M), int(K), dens_a, dup_prob=0.2)
    B = random_csr(rng, int(K), int(N), dens_b, dup_prob=0.2)
    Ad, Bd = to_count_dense(A), to_count_dense(B)
    # FLOP: every stored A(i,k) meets every stored entry of B row k
    flop_bf = Ad @ Bd.sum(axis=1)
    # exact structure: boolean OR-AND product
    nnz_bf = ((Ad > 0).astype(np.int64) @ (Bd > 0).astype(np.int64) > 0).sum(axis=1)
    rf, F = oracle_mod.row_flop(A, B)
    assert np.array_equal(rf.astype(np.int64), flop_bf)
    assert F == int(flop_bf.sum())
    ex, st = oracle_mod.exact(A, B)
    assert np.array_equal(ex, nnz_bf)
    assert st.out_sum == int(nnz_bf.sum()) and st.total_flop == F
    sub = np.array([0, int(M) - 1, int(M) // 2], dtype=np.int32)
    nz, rf2 = oracle_mod.rows_nnz(A, B, sub)
    assert np.array_equal(nz, nnz_bf[sub]) and np.array_equal(rf2.astype(np.int64), flop_bf[sub])


@pytest.mark.parametrize("seed", range(6))
def test_sampled_sums_vs_brute_force(oracle_mod, seed):
    # f* and z* are the brute-force FLOP and NNZ summed over the sampled rows
    rng = np.random.default_rng(100 + seed)
    A = random_csr(rng, 60, 30, 0.15, dup_prob=0.1)
    B = random_csr(rng, 30, 25, 0.2, dup_prob=0.1)
    Ad, Bd = to_count_dense(A), to_count_dense(B)
    flop_bf = Ad @ Bd.sum(axis=1)
    nnz_bf = ((Ad > 0).astype(np.int64) @ (Bd > 0).astype(np.int64) > 0).sum(axis=1)
    for rate, mode in ((0.3, oracle_mod.BERNOULLI), (1.0, oracle_mod.BERNOULLI)):
        S = oracle_mod.sample_rows(A.nrows, rate, seed, mode)
        _, _, st = oracle_mod.predict(A, B, rate, seed, mode)
        assert st.n_sampled == S.size
        assert st.sample_flop == int(flop_bf[S].sum())
        assert st.sample_nnz == int(nnz_bf[S].sum())


# ------------------------------------------------------- closed forms

def _stencil_1d(n):
    # 1-D 3-point pattern T; the 27-point stencil is T (x) T (x) T in natural
    # order, so A^2 = T^2 (x) T^2 (x) T^2 and both the row FLOP and the row NNZ
    # of A^2 are products of 1-D factors over the three grid coordinates
    deg = np.array([1 + (x > 0) + (x < n - 1) for x in range(n)])
    s = np.array([sum(deg[k] for k in range(max(0, x - 1), min(n, x + 2))) for x in range(n)])
    c = np.array([1 + min(x, 2) + min(n - 1 - x, 2) for x in range(n)])
    return deg, s, c


@pytest.mark.parametrize("n", [4, 7, 12])
def test_stencil27_closed_form_row_by_row(oracle_mod, n):
    A = workloads.stencil27(n)
    deg, s, c = _stencil_1d(n)
    r = np.arange(n ** 3)
    x, y, z = r % n, (r // n) % n, r // (n * n)
    assert np.array_equal(A.row_lengths(), deg[x] * deg[y] * deg[z])
    rf, F = oracle_mod.row_flop(A, A)
    assert np.array_equal(rf.astype(np.int64), s[x] * s[y] * s[z])
    ex, st = oracle_mod.exact(A, A)
    assert np.array_equal(ex, c[x] * c[y] * c[z])
    assert F == (9 * n - 10) ** 3 and st.out_sum == (5 * n - 6) ** 3


def test_stencil128_totals(oracle_mod):
    A = workloads.stencil27(128)
    assert A.nnz == 382 ** 3 == 55_742_968
    rf, F = oracle_mod.row_flop(A, A)
    assert F == 1142 ** 3 == 1_489_355_288
    assert int(rf.max()) == 729


def test_uniform4096_row_flop_is_constant(oracle_mod):
    w = workloads.uniform4096()
    rf, F = oracle_mod.row_flop(w.A, w.B)
    assert np.all(rf == 64) and F == 2 ** 18


def test_stencil_times_uniform_row_flop(oracle_mod):
    A = workloads.stencil27(10)
    B = workloads.uniform(A.ncols, 4096, 4, 1)
    rf, F = oracle_mod.row_flop(A, B)
    assert np.array_equal(rf.astype(np.int64), 4 * A.row_lengths()) and F == 4 * A.nnz


def test_identity_and_permutation(oracle_mod):
    rng = np.random.default_rng(5)
    B = random_csr(rng, 50, 40, 0.2, dup_prob=0.0)
    I = from_rows([[i] for i in range(50)], 50)
    ex, _ = oracle_mod.exact(I, B)
    assert np.array_equal(ex, B.row_lengths())
    # a permutation A gives CR = 1: the prediction equals the row FLOP
    perm = rng.permutation(50)
    P = from_rows([[int(p)] for p in perm], 50)
    for rate in (0.3, 1.0):
        pred, rf, st = oracle_mod.predict(P, B, rate, 11)
        if st.sample_flop:
            assert np.array_equal(pred, rf.astype(np.int64))


def test_identical_B_rows_predict_exactly(oracle_mod):
    # every B row holds the same L distinct columns and every A row names a
    # distinct B rows: row FLOP = a L, row NNZ = L, CR = a for every row and for
    # every sample, so every prediction is exactly L
    L, a, K = 7, 5, 40
    rng = np.random.default_rng(9)
    cols = sorted(rng.choice(100, size=L, replace=False).tolist())
    B = from_rows([cols] * K, 100)
    A = from_rows([sorted(rng.choice(K, size=a, replace=False).tolist()) for _ in range(300)], K)
    for rate, seed in ((0.05, 1), (0.5, 2), (1.0, 3)):
        pred, rf, st = oracle_mod.predict(A, B, rate, seed)
        assert st.sample_flop > 0
        assert np.all(rf == a * L) and np.all(pred == L)


# ---------------------------------------------------------- worked example

def _worked():
    with open(os.path.join(GOLDEN, "worked_example.json")) as f:
        return json.load(f)


def test_worked_example_full(oracle_mod):
    w = _worked()
    B = from_rows(w["B"]["rows"], w["B"]["ncols"])
    A = from_rows(w["A_full"]["rows"], w["A_full"]["ncols"])
    e = w["A_full_expect"]
    rf, F = oracle_mod.row_flop(A, B)
    assert rf.tolist() == e["row_flop"] and F == e["F"]
    ex, st = oracle_mod.exact(A, B)
    assert ex.tolist() == e["nnz_exact"] and st.out_sum == e["Z"]
    pred, _, st = oracle_mod.predict(A, B, 1.0, 123)
    r1 = e["rate1"]
    assert (st.n_sampled, st.sample_flop, st.sample_nnz) == (r1["n_s"], r1["f_star"], r1["z_star"])
    assert pred.tolist() == r1["nnz_pred"] and st.out_sum == r1["pred_sum"]
    assert st.z2_star == Fraction(*r1["z2_star"])
    ref, _ = oracle_mod.reference(A, B, 1.0, 123)
    assert ref.tolist() == r1["nnz_ref"]
    pred, _, st = oracle_mod.predict(A, B, 0.0, 123)
    assert pred.tolist() == e["rate0"]["nnz_pred"]
    assert st.n_sampled == 0 and (st.flags & oracle_mod.FLAG_EMPTY_SAMPLE)


def test_worked_example_partial_sample(oracle_mod):
    w = _worked()
    B = from_rows(w["B"]["rows"], w["B"]["ncols"])
    A = from_rows(w["A_three"]["rows"], w["A_three"]["ncols"])
    e = w["A_three_seed0_rate_half"]
    assert oracle_mod.sample_rows(3, 0.5, 0).tolist() == e["sampled_rows"]
    pred, _, st = oracle_mod.predict(A, B, 0.5, 0)
    assert (st.total_flop, st.n_sampled, st.sample_flop, st.sample_nnz) == \
        (e["F"], e["n_s"], e["f_star"], e["z_star"])
    assert pred.tolist() == e["nnz_pred"]
    ref, st_r = oracle_mod.reference(A, B, 0.5, 0)
    assert ref.tolist() == e["nnz_ref"]
    assert st.z2_star == Fraction(*e["z2_star"]) and st.z1_star == Fraction(*e["z1_star"])
    assert st.f_star == Fraction(*e["f_star_est"])
    err = oracle_mod.relative_errors(st, e["Z"])
    assert err["eps1"] == Fraction(*e["eps1"])
    assert err["epsf"] == Fraction(*e["epsf"])
    assert err["eps2"] == Fraction(*e["eps2"])


# ----------------------------------------------------------- invariants

def _some_cases():
    rng = np.random.default_rng(77)
    out = []
    for s in range(8):
        A = random_csr(rng, 120, 60, rng.uniform(0.01, 0.2), dup_prob=0.1)
        B = random_csr(rng, 60, 50, rng.uniform(0.01, 0.3), dup_prob=0.1)
        out.append((A, B))
    for st in ("uniform", "rmat", "banded", "blockdiag", "zipf"):
        A = workloads.make(st, 2048, 4, 1)
        out.append((A, A))
    return out


@pytest.mark.parametrize("rate", [0.02, 0.2, 1.0])
def test_invariants(oracle_mod, rate):
    for A, B in _some_cases():
        rf, F = oracle_mod.row_flop(A, B)
        ex, st_e = oracle_mod.exact(A, B)
        Z = st_e.out_sum
        rf_i = rf.astype(np.int64)
        # nnz_i <= min(row_flop_i, N)
        assert np.all(ex <= np.minimum(rf_i, B.ncols))
        # sum of row FLOP = sum_k colcount_A(k) * rowlen_B(k)
        colcount = np.bincount(A.col, minlength=A.ncols)
        assert F == int(np.dot(colcount.astype(np.int64), B.row_lengths()))
        pred, rf2, st = oracle_mod.predict(A, B, rate, 4242)
        assert np.array_equal(rf2, rf) and st.total_flop == F
        S = oracle_mod.sample_rows(A.nrows, rate, 4242)
        assert st.sample_nnz <= st.sample_flop
        assert st.sample_nnz >= int(np.sum(rf_i[S] > 0))
        if st.sample_flop:
            assert np.all(pred <= rf_i)
            assert np.array_equal(pred == 0, rf_i == 0)
            # Eq. (4): the per-row predictions sum to Z2* up to the ceilings
            z2 = st.z2_star
            assert z2 <= st.out_sum < z2 + int(np.sum(rf_i > 0)) + 1
            ref, st_r = oracle_mod.reference(A, B, rate, 4242)
            z1 = st_r.z1_star
            assert z1 <= st_r.out_sum < z1 + int(np.sum(rf_i > 0)) + 1
            err = oracle_mod.relative_errors(st, Z)
            if err["eps1"] is not None and err["epsf"] is not None:
                # Eq. (5), exactly in rationals
                assert (1 + err["eps2"]) * (1 + err["epsf"]) == 1 + err["eps1"]
        if rate == 1.0:
            assert st.n_sampled == A.nrows and st.sample_flop == F and st.sample_nnz == Z
            assert st.z2_star == Z
            ref, st_r = oracle_mod.reference(A, B, rate, 4242)
            assert st_r.z1_star == Z and np.array_equal(ref, pred)


def test_paper_sampler_mode(oracle_mod):
    # Sec. V-B sampler: min(floor(0.003 M), 300) draws with replacement
    A = workloads.uniform(50_000, 50_000, 3, 2)
    S = oracle_mod.sample_rows(A.nrows, 0.0, 9, oracle_mod.PAPER)
    assert S.size == 150 and S.min() >= 0 and S.max() < A.nrows
    _, _, st = oracle_mod.predict(A, A, 0.0, 9, oracle_mod.PAPER)
    nz, rf = oracle_mod.rows_nnz(A, A, S)
    assert st.n_sampled == 150
    assert st.sample_flop == int(rf.astype(np.int64).sum())  # duplicates count per draw
    assert st.sample_nnz == int(nz.sum())
    assert oracle_mod.paper_sample_num(333) == 0 and oracle_mod.paper_sample_num(10**6) == 300
    _, _, st = oracle_mod.predict(workloads.uniform(200, 200, 2, 1),
                                  workloads.uniform(200, 200, 2, 1), 0.0, 1, oracle_mod.PAPER)
    assert st.n_sampled == 0 and st.flags & oracle_mod.FLAG_EMPTY_SAMPLE


def test_paper_sampler_known_rows(oracle_mod):
    # Alg. 2 and Sec. V-B: draw r picks row floor(M u_r).  Known answers worked
    # by hand from the published first outputs of splitmix64 from state 0
    # (golden/worked_example.json): they fix the draw -> row mapping (floor of
    # M u, not u mod M, not a rounding) and the stream (seed, counter from 0).
    ex = json.load(open(os.path.join(GOLDEN, "worked_example.json")))["paper_sampler_seed0"]
    S = oracle_mod.sample_rows(1000, 0.0, 0, oracle_mod.PAPER)
    assert S.tolist() == ex["M1000"]["rows"]
    S = oracle_mod.sample_rows(46835, 0.0, 0, oracle_mod.PAPER)
    assert S.size == ex["M46835"]["sample_num"]
    assert S[:3].tolist() == ex["M46835"]["first_rows"]
    # every draw, by exact rational arithmetic on the pinned generator outputs:
    # row = floor(M * (x >> 11) / 2^53), which lies in [0, M) for any x
    for M, seed in ((46835, 0), (100_000, 1001), (2**31 - 1, 7), (334, 2**64 - 1)):
        S = oracle_mod.sample_rows(M, 0.0, seed, oracle_mod.PAPER)
        assert S.size == oracle_mod.paper_sample_num(M)
        for r, row in enumerate(S.tolist()):
            u = Fraction(oracle_mod.splitmix64(seed, r) >> 11, 2**53)
            assert row == math.floor(M * u) and 0 <= row < M


def test_reference_wide_division(oracle_mod):
    # Eq. (2) per row: ceil(rf z* M / (n_s F)).  Its quotient is at most M N <
    # 2^62 but the numerator reaches 2^155 under the int32 CSR format (rf <
    # 2^62, z* M < 2^93), so the oracle divides a 192-bit product; checked
    # against Python's exact integers, at the format's extremes too.
    rng = np.random.default_rng(11)
    cases = [(1, 1, 1), (5, 12, 17), (2**62 - 1, (2**62 - 1) * (2**31 - 1), 2**31 * (2**62 - 1)),
             (2**62 - 1, 2**93 - 1, 2**93 - 1), (3, 2**64 + 5, 7)]
    for _ in range(2000):
        a = int(rng.integers(1, 2**62))
        d = int(rng.integers(1, 2**62)) * int(rng.integers(1, 2**31))
        qmax = (d << 64) // a  # keep the quotient below 2^64
        q = int(rng.integers(0, 2**62)) * int(rng.integers(1, 2**31)) % max(qmax, 1)
        cases.append((a, q, d))
    wide = 0
    for a, q, d in cases:
        assert oracle_mod.ceil_mul_div_wide(a, q, d) == -(-(a * q) // d), (a, q, d)
        wide += a * q >= 2**128
    assert wide > 100  # the 192-bit branch is exercised


def test_check_csr(oracle_mod):
    A = workloads.uniform(100, 50, 5, 1)
    assert oracle_mod.check_csr(A) == 0
    bad = workloads.CSR(A.nrows, A.ncols, A.rpt.copy(), A.col.copy())
    bad.col[3] = 50
    assert oracle_mod.check_csr(bad) != 0
