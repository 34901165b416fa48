"""GPU path == CPU oracle, bit for bit, through the C ABI.

Every output of the HIP library is an integer, so the bar is exact equality of
every element and of every statistics field.  Small cases span several tiles
of the streaming kernel (256..2048 rows each), every symbolic bin and its
boundaries, split long rows and multi-window bitmaps, with ragged tails; the
full-size workloads run in the launch configuration the benchmark times.
"""
import ctypes
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from tests.csr_util import from_rows, random_csr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
STAT_KEYS = ("total_flop", "n_sampled", "sample_flop", "sample_nnz", "out_sum", "nrows", "flags",
             "a_sample_nnz")


@pytest.fixture(scope="module")
def ssp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2207_13848_amd as m
    return m


def _dev(ssp, M):
    return ssp.DeviceCSR.from_csr(M, "cuda:0")


def _say(msg):
    print(msg, flush=True)


def _check_stats(gpu_st, o_st, what):
    for k in STAT_KEYS:
        assert gpu_st[k] == getattr(o_st, k), f"{what}: stats.{k} gpu={gpu_st[k]} " \
                                              f"oracle={getattr(o_st, k)}"


def check_predict(ssp, A, B, rate, seed, sampler="bernoulli", Ad=None, Bd=None):
    mode = oracle.PAPER if sampler == "paper" else oracle.BERNOULLI
    Ad = Ad if Ad is not None else _dev(ssp, A)
    Bd = Bd if Bd is not None else (Ad if B is A else _dev(ssp, B))
    pred, rf, st = ssp.predict_structure(Ad, Bd, rate, seed, sampler=sampler,
                                         return_row_flop=True)
    torch.cuda.synchronize()
    o_pred, o_rf, o_st = oracle.predict(A, B, rate, seed, mode)
    assert np.array_equal(rf.cpu().numpy(), o_rf.astype(np.int64)), "row_flop"
    assert np.array_equal(pred.cpu().numpy(), o_pred), "nnz_pred"
    _check_stats(ssp.read_stats(st), o_st, "predict")
    return o_st


def check_reference(ssp, A, B, rate, seed, sampler="bernoulli", Ad=None, Bd=None):
    mode = oracle.PAPER if sampler == "paper" else oracle.BERNOULLI
    Ad = Ad if Ad is not None else _dev(ssp, A)
    Bd = Bd if Bd is not None else (Ad if B is A else _dev(ssp, B))
    ref, st = ssp.reference_estimate(Ad, Bd, rate, seed, sampler=sampler)
    torch.cuda.synchronize()
    o_ref, o_st = oracle.reference(A, B, rate, seed, mode)
    assert np.array_equal(ref.cpu().numpy(), o_ref), "nnz_ref"
    _check_stats(ssp.read_stats(st), o_st, "reference")


def _exact_golden(name):
    """The oracle's every-row exact structure of a full-size product, as
    written by tests/golden/make_exact_oracle.py (Z, F, SHA-256 of nnz_exact
    as little-endian int64)."""
    with open(os.path.join(GOLDEN, "exact_oracle.json")) as f:
        return json.load(f)[name]


def check_exact(ssp, A, B, Ad=None, Bd=None, full_limit=10 ** 8, golden=None):
    """Every row when the serial oracle can afford it (F <= full_limit), or
    against the stored digest of the oracle's every-row result (`golden`);
    else (and besides) the 40 longest rows and 2000 random rows one by one
    plus F and the sum."""
    Ad = Ad if Ad is not None else _dev(ssp, A)
    Bd = Bd if Bd is not None else (Ad if B is A else _dev(ssp, B))
    ex, st = ssp.exact_structure(Ad, Bd)
    torch.cuda.synchronize()
    ex = ex.cpu().numpy()
    if golden is not None:
        g = _exact_golden(golden)
        assert g["nrows"] == A.nrows and g["nnz_A"] == A.nnz and g["nnz_B"] == B.nnz
        s = ssp.read_stats(st)
        assert s["out_sum"] == g["Z"] and s["total_flop"] == g["F"], "Z or F != oracle"
        digest = hashlib.sha256(np.ascontiguousarray(ex, dtype="<i8").tobytes()).hexdigest()
        assert digest == g["nnz_exact_sha256"], "nnz_exact differs from the oracle's rows"
    rf, F = oracle.row_flop(A, B)
    if F <= full_limit:
        o_ex, o_st = oracle.exact(A, B)
        assert np.array_equal(ex, o_ex), "nnz_exact"
        _check_stats(ssp.read_stats(st), o_st, "exact")
        return
    rng = np.random.default_rng(0)
    rows = np.unique(np.concatenate([np.argsort(rf)[-40:],
                                     rng.integers(0, A.nrows, 2000)])).astype(np.int32)
    o_nnz, _ = oracle.rows_nnz(A, B, rows)
    assert np.array_equal(ex[rows], o_nnz), "nnz_exact (sampled rows)"
    s = ssp.read_stats(st)
    assert s["total_flop"] == F and s["out_sum"] == int(ex.sum())
    assert np.all(ex <= np.minimum(rf.astype(np.int64), B.ncols))


def check_all(ssp, A, B, rate, seed):
    Ad = _dev(ssp, A)
    Bd = Ad if B is A else _dev(ssp, B)
    check_predict(ssp, A, B, rate, seed, Ad=Ad, Bd=Bd)
    check_reference(ssp, A, B, rate, seed, Ad=Ad, Bd=Bd)
    check_exact(ssp, A, B, Ad=Ad, Bd=Bd)


# ------------------------------------------------------------ worked example

def test_worked_example_on_gpu(ssp):
    w = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    B = from_rows(w["B"]["rows"], w["B"]["ncols"])
    A = from_rows(w["A_full"]["rows"], w["A_full"]["ncols"])
    Ad, Bd = _dev(ssp, A), _dev(ssp, B)
    e = w["A_full_expect"]
    pred, rf, st = ssp.predict_structure(Ad, Bd, 1.0, 123, return_row_flop=True)
    assert rf.cpu().tolist() == e["row_flop"]
    assert pred.cpu().tolist() == e["rate1"]["nnz_pred"]
    ex, st = ssp.exact_structure(Ad, Bd)
    assert ex.cpu().tolist() == e["nnz_exact"] and ssp.read_stats(st)["out_sum"] == e["Z"]
    pred, _, st = ssp.predict_structure(Ad, Bd, 0.0, 123)
    assert pred.cpu().tolist() == e["rate0"]["nnz_pred"]
    assert ssp.read_stats(st)["flags"] & ssp.FLAG_EMPTY_SAMPLE
    A3 = _dev(ssp, from_rows(w["A_three"]["rows"], w["A_three"]["ncols"]))
    e3 = w["A_three_seed0_rate_half"]
    pred, _, st = ssp.predict_structure(A3, Bd, 0.5, 0)
    assert pred.cpu().tolist() == e3["nnz_pred"]
    s = ssp.read_stats(st)
    assert (s["n_sampled"], s["sample_flop"], s["sample_nnz"]) == (e3["n_s"], e3["f_star"],
                                                                   e3["z_star"])
    ref, _ = ssp.reference_estimate(A3, Bd, 0.5, 0)
    assert ref.cpu().tolist() == e3["nnz_ref"]


# ------------------------------------------------------------ random small

@pytest.mark.parametrize("seed", range(10))
def test_random_small_with_duplicates_and_unsorted_rows(ssp, seed):
    rng = np.random.default_rng(1000 + seed)
    M, K, N = (int(x) for x in rng.integers(1, 300, size=3))
    A = random_csr(rng, M, K, float(rng.uniform(0.0, 0.15)), dup_prob=0.2)
    B = random_csr(rng, K, N, float(rng.uniform(0.0, 0.3)), dup_prob=0.2)
    _say(f"random seed={seed} M={M} K={K} N={N} nnzA={A.nnz} nnzB={B.nnz}")
    for rate in (0.0, 0.1, 0.5, 1.0):
        check_predict(ssp, A, B, rate, 7 * seed + 1)
    check_reference(ssp, A, B, 0.3, seed)
    check_exact(ssp, A, B)


@pytest.mark.parametrize("structure", workloads.STRUCTURES)
@pytest.mark.parametrize("n,d", [(1000, 2), (5003, 8), (70001, 32)])
def test_generator_families(ssp, structure, n, d):
    A = workloads.make(structure, n, d, 3)
    _say(f"family {structure} n={n} d={d} nnz={A.nnz}")
    check_all(ssp, A, A, 0.05, 77)


def test_paper_sampler(ssp):
    A = workloads.rmat(200_000, 8, 2)
    _say(f"paper sampler rmat n={A.nrows}")
    check_predict(ssp, A, A, 0.0, 5, sampler="paper")
    check_reference(ssp, A, A, 0.0, 5, sampler="paper")
    small = workloads.uniform(300, 300, 3, 1)  # 0.003 * 300 < 1: no draws
    st = check_predict(ssp, small, small, 0.0, 5, sampler="paper")
    assert st.n_sampled == 0


# ------------------------------------------------------------ edge cases

def test_degenerate_shapes(ssp):
    empty_rows = workloads.CSR(0, 5, np.zeros(1, np.int32), np.zeros(0, np.int32))
    B = workloads.uniform(5, 7, 2, 1)
    pred, _, st = ssp.predict_structure(_dev(ssp, empty_rows), _dev(ssp, B), 0.5, 1)
    assert pred.numel() == 0 and ssp.read_stats(st)["total_flop"] == 0
    ex, _ = ssp.exact_structure(_dev(ssp, empty_rows), _dev(ssp, B))
    assert ex.numel() == 0
    # K = 0: A is M x 0, B is 0 x N
    A0 = workloads.CSR(9, 0, np.zeros(10, np.int32), np.zeros(0, np.int32))
    B0 = workloads.CSR(0, 4, np.zeros(1, np.int32), np.zeros(0, np.int32))
    check_all(ssp, A0, B0, 0.5, 3)
    # N = 0: every B row empty -> no products, empty-sample fallback
    A1 = workloads.uniform(50, 20, 3, 1)
    B1 = workloads.CSR(20, 0, np.zeros(21, np.int32), np.zeros(0, np.int32))
    check_all(ssp, A1, B1, 1.0, 3)
    # nnz(A) = 0 with K > 0
    A2 = workloads.CSR(33, 20, np.zeros(34, np.int32), np.zeros(0, np.int32))
    check_all(ssp, A2, workloads.uniform(20, 30, 4, 2), 1.0, 3)
    # a single row
    A3 = from_rows([[0, 3, 3, 1]], 5)
    check_all(ssp, A3, workloads.uniform(5, 9, 3, 4), 1.0, 3)


def test_bin_boundaries(ssp):
    # rows whose product counts sit on both sides of every bin edge; B rows of
    # length 1 make row FLOP = row length of A
    K = 20000
    B = workloads.uniform(K, 50000, 1, 5)
    sizes = [1, 2, 63, 64, 65, 127, 128, 129, 255, 256, 257, 1023, 1024, 1025, 4096, 8191, 8192,
             8193, 9000, 16384, 17000]
    rng = np.random.default_rng(5)
    rows = [sorted(rng.choice(K, size=s, replace=False).tolist()) for s in sizes]
    A = from_rows(rows * 3, K)
    _say("bin boundaries")
    check_all(ssp, A, B, 1.0, 11)
    check_all(ssp, A, B, 0.4, 12)


def _copies_case(n, kinds):
    # for every length L in 1..n, B holds c identical rows {0..L-1} for the
    # largest c in `kinds`, and A a row naming k of them for every k in
    # `kinds`: k L products, L distinct columns
    c = max(kinds)
    brows, arows = [], []
    for L in range(1, n + 1):
        base = len(brows)
        brows += [list(range(L))] * c
        arows += [list(range(base, base + k)) for k in kinds]
    return from_rows(arows, len(brows)), from_rows(brows, n)


@pytest.mark.parametrize("kinds,num,den", [((4, 2), 1, 3), ((10,), 1, 10), ((7, 3, 3), 3, 13)])
def test_prediction_ceiling_at_whole_quotients(ssp, kinds, num, den):
    # At rate 1 the sampled ratio z*/f* is num/den exactly (kinds (4, 2):
    # 2S columns over 6S products), so a row of rf products is predicted
    # ceil(rf num / den), a whole quotient whenever den divides rf num, where
    # the double nearest num/den lies a little below (1/3) or above (1/10).
    A, B = _copies_case(300, kinds)
    _say(f"whole quotients {kinds}")
    Ad, Bd = _dev(ssp, A), _dev(ssp, B)
    st = check_predict(ssp, A, B, 1.0, 3, Ad=Ad, Bd=Bd)
    assert st.sample_nnz * den == st.sample_flop * num
    pred, rf, _ = ssp.predict_structure(Ad, Bd, 1.0, 3, return_row_flop=True)
    rf = rf.cpu().numpy()
    assert np.array_equal(pred.cpu().numpy(), -((-rf * num) // den))
    assert np.any(rf * num % den == 0)
    check_predict(ssp, A, B, 0.5, 4, Ad=Ad, Bd=Bd)
    # the same ceilings by the 128-bit division (rows of 2^48 or more
    # products take it by default; a tuning sends every row there)
    h = ssp.Handle(0)
    ssp.set_tuning(dict(ssp.default_tuning(), est_max_rf=0), handle=h)
    pred2, _, _ = ssp.predict_structure(Ad, Bd, 1.0, 3, handle=h)
    torch.cuda.synchronize()
    assert np.array_equal(pred2.cpu().numpy(), -((-rf * num) // den))
    h.close()


def _long_rows(ncols, nbig, seed):
    # long rows whose entries name B rows of all three length classes the
    # long-row kernel treats differently: huge (>= 2048 entries), medium
    # (walked in units: at least the tuning's long_len, 16 by default) and
    # short (flattened; lengths 0..19 here); the largest rows exceed the default split
    # threshold (2^19 products) more than twice over
    rng = np.random.default_rng(seed)
    K = 3000
    brows = []
    for k in range(K):
        if k < 400:
            L = 3000
        elif k < 700:
            L = int(rng.integers(32, 1500))
        else:
            L = int(rng.integers(0, 20))
        brows.append(sorted(rng.choice(ncols, size=L, replace=False).tolist()))
    B = from_rows(brows, ncols)
    arows = []
    for i in range(400):
        if i % (400 // nbig) == 0:
            hubs = rng.choice(400, size=int(rng.integers(20, 400)), replace=False).tolist()
            meds = (400 + rng.choice(300, size=150, replace=False)).tolist()
            arows.append(hubs + meds + rng.choice(K, size=500, replace=False).tolist())
        elif i % 7 == 0:
            arows.append((400 + rng.choice(300, size=40, replace=False)).tolist())
        else:
            arows.append(rng.choice(K, size=int(rng.integers(0, 30)), replace=False).tolist())
    return from_rows(arows, K), B


def test_split_long_rows(ssp):
    A, B = _long_rows(300_000, 8, 1)
    rf, _ = oracle.row_flop(A, B)
    assert rf.max() > 2 * 2 ** 19
    _say(f"split long rows max rf={rf.max()}")
    check_all(ssp, A, B, 1.0, 1)
    check_all(ssp, A, B, 0.3, 2)


def test_rows_of_many_entries_and_few_products(ssp):
    # long rows (bin 4) with more entries than one 1024-entry chunk but few
    # products (short B rows): split by chunks although far below the split
    # target; among them ordinary light long rows, so the parts and the light
    # list meet in the bin-4 list
    rng = np.random.default_rng(11)
    K, N = 20000, 1 << 20
    brows = [sorted(rng.choice(N, size=int(rng.integers(1, 6)), replace=False).tolist())
             for _ in range(K)]
    B = from_rows(brows, N)
    arows = []
    for i in range(300):
        if i % 10 == 0:  # 1025..4000 entries: two to four chunks
            arows.append(rng.choice(K, size=int(rng.integers(1025, 4000)), replace=False).tolist())
        elif i % 10 == 1:  # light long rows: a few hundred entries
            arows.append(rng.choice(K, size=int(rng.integers(400, 900)), replace=False).tolist())
        else:
            arows.append(rng.choice(K, size=int(rng.integers(0, 40)), replace=False).tolist())
    A = from_rows(arows, K)
    rf, _ = oracle.row_flop(A, B)
    alen = np.diff(A.rpt)
    assert (alen > 1024).sum() >= 20 and rf.max() < 2 ** 17
    _say(f"many-entry rows: max len {alen.max()} max rf {rf.max()}")
    check_all(ssp, A, B, 1.0, 5)
    check_all(ssp, A, B, 0.5, 6)


def test_long_rows_over_several_bitmap_windows(ssp):
    # N > 2^20 columns: the long-row bitmap covers the columns in windows
    A, B = _long_rows((1 << 21) + 12345, 5, 2)
    _say("multi-window long rows")
    check_all(ssp, A, B, 1.0, 3)


def test_widest_b(ssp):
    # B with 2^31 - 1 columns, the largest 32-bit column count: columns at
    # both ends of the range, short rows hashed over the whole range, and a
    # few long rows whose bitmap walks 2048 windows of 2^20 columns
    N = 2 ** 31 - 1
    rng = np.random.default_rng(9)
    K = 400
    brows = []
    for k in range(K):
        L = 3000 if k < 8 else int(rng.integers(0, 40))
        cols = set(int(c) for c in rng.integers(0, N, L))
        if k % 5 == 0:
            cols |= {0, N - 1, N - 2, (1 << 20) - 1, 1 << 20}
        brows.append(sorted(cols))
    B = from_rows(brows, N)
    arows = [list(range(8)) + rng.choice(K, 20, replace=False).tolist() for _ in range(3)]
    arows += [rng.choice(np.arange(8, K), int(rng.integers(0, 30)), replace=False).tolist()
              for _ in range(297)]
    A = from_rows(arows, K)
    rf, _ = oracle.row_flop(A, B)
    assert rf.max() > 8192 and B.col.max() == N - 1
    _say("widest B")
    check_all(ssp, A, B, 1.0, 1)
    check_all(ssp, A, B, 0.3, 2)


def test_b_with_more_than_2_30_rows(ssp):
    # K = 2^30 + 5 rows of B (a 4 GiB row-pointer array): beyond the 32-bit
    # byte offsets of the streaming kernel's buffer loads, so it takes its
    # other form; A's entries name rows at both ends of the range
    K = (1 << 30) + 5
    N = 5000
    rng = np.random.default_rng(12)
    ks = np.unique(np.concatenate([rng.integers(0, K, 3000), [0, 1, K - 1, K - 2, 1 << 30,
                                                              (1 << 30) - 1]])).astype(np.int64)
    lens = rng.integers(0, 60, ks.shape[0])
    lens[ks == K - 1] = 3000  # one long B row: the long-row kernel too
    rpt = np.zeros(K + 1, dtype=np.int32)
    ends = np.cumsum(lens)
    for j in range(ks.shape[0]):  # rpt[i] = products of rows below i
        rpt[ks[j] + 1: (ks[j + 1] + 1 if j + 1 < ks.shape[0] else K + 1)] = ends[j]
    col = np.concatenate([np.sort(rng.choice(N, int(L), replace=False)) for L in lens]
                         ).astype(np.int32)
    B = workloads.CSR(K, N, rpt, col, "b_2_30_rows")
    arows = [rng.choice(ks, int(rng.integers(0, 40)), replace=False).tolist() for _ in range(1500)]
    arows[7] = ks.tolist()[:300] + [K - 1]
    A = from_rows(arows, K)
    _say(f"B with {K} rows")
    Ad, Bd = _dev(ssp, A), _dev(ssp, B)
    check_predict(ssp, A, B, 0.3, 5, Ad=Ad, Bd=Bd)
    check_reference(ssp, A, B, 0.3, 5, Ad=Ad, Bd=Bd)
    check_exact(ssp, A, B, Ad=Ad, Bd=Bd)
    del Bd
    torch.cuda.empty_cache()


def test_misaligned_column_array(ssp):
    # a column array that is not 16-byte aligned (the streaming kernel's
    # buffer loads take it as it is)
    A = workloads.zipf(20000, 8, 4)
    big = torch.zeros(A.nnz + 1, dtype=torch.int32, device="cuda:0")
    big[1:] = torch.as_tensor(A.col, device="cuda:0")
    Ad = ssp.DeviceCSR(torch.as_tensor(A.rpt, device="cuda:0"), big[1:], A.ncols)
    assert Ad.col.data_ptr() % 16 != 0
    _say("misaligned col")
    Bd = _dev(ssp, A)
    check_predict(ssp, A, A, 0.1, 9, Ad=Ad, Bd=Bd)
    check_exact(ssp, A, A, Ad=Ad, Bd=Bd)


@pytest.mark.parametrize("M", [256 * 2048, 256 * 2048 + 1])
def test_sampling_scan_with_and_without_its_own_launch(ssp, M):
    # 2048 candidates per sampling group: 256 groups (the write pass scans the
    # group counts itself) and 257 (a scan launch of its own)
    A = workloads.uniform(M, 4096, 2, 6)
    B = workloads.uniform(4096, 4096, 4, 7)
    _say(f"sampling groups M={M}")
    Ad, Bd = _dev(ssp, A), _dev(ssp, B)
    check_predict(ssp, A, B, 0.01, 21, Ad=Ad, Bd=Bd)
    check_predict(ssp, A, B, 0.7, 22, Ad=Ad, Bd=Bd)
    check_reference(ssp, A, B, 0.01, 23, Ad=Ad, Bd=Bd)


def test_repeat_calls_are_identical(ssp):
    A = workloads.rmat(1 << 16, 16, 9)
    Ad = _dev(ssp, A)
    outs = []
    for _ in range(3):
        p, _, st = ssp.predict_structure(Ad, Ad, 0.02, 5)
        outs.append((p.clone(), st.clone()))
    torch.cuda.synchronize()
    for p, st in outs[1:]:
        assert torch.equal(p, outs[0][0]) and torch.equal(st, outs[0][1])


def test_non_default_stream(ssp):
    A = workloads.banded(30000, 16, 2)
    Ad = _dev(ssp, A)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        p, _, st = ssp.predict_structure(Ad, Ad, 0.05, 3)
    s.synchronize()
    o_pred, _, _ = oracle.predict(A, A, 0.05, 3)
    assert np.array_equal(p.cpu().numpy(), o_pred)


# ------------------------------------------------------------ errors

def test_host_side_errors(ssp):
    from paper_2207_13848_amd import _native
    lib = _native.load()
    h = ssp.default_handle("cuda:0")
    A = _dev(ssp, workloads.uniform(100, 60, 3, 1))
    B = _dev(ssp, workloads.uniform(60, 40, 3, 1))
    out = torch.empty(100, dtype=torch.int64, device="cuda:0")
    a, b = A._c(), B._c()
    call = lambda aa, bb, rate, o: lib.ssp_predict_structure(  # noqa: E731
        h.ptr, ctypes.byref(aa), ctypes.byref(bb), rate, 1, o, None, None, None)
    assert call(a, b, 0.5, out.data_ptr()) == 0
    assert call(b, a, 0.5, out.data_ptr()) == -2            # 40 != 100
    assert call(a, b, float("nan"), out.data_ptr()) == -1
    assert call(a, b, 1.5, out.data_ptr()) == -1
    assert call(a, b, -0.1, out.data_ptr()) == -1
    assert call(a, b, 0.5, None) == -1
    neg = _native.SspCsr(-1, 60, 0, A.rpt.data_ptr(), A.col.data_ptr())
    assert call(neg, b, 0.5, out.data_ptr()) == -1
    big = _native.SspCsr(100, 60, 1 << 31, A.rpt.data_ptr(), A.col.data_ptr())
    assert call(big, b, 0.5, out.data_ptr()) == -3
    assert lib.ssp_predict_structure_ex(h.ptr, ctypes.byref(a), ctypes.byref(b), 7, 0.5, 1,
                                        out.data_ptr(), None, None, None) == -1
    torch.cuda.synchronize()
    # a handle with a tiny budget refuses to grow its workspace
    tiny = ssp.Handle(0, hbm_budget_bytes=4096)
    with pytest.raises(ssp.SspError) as ei:
        ssp.predict_structure(A, B, 0.5, 1, handle=tiny)
    assert ei.value.status == -4
    tiny.close()


def test_validate_csr(ssp):
    A = workloads.uniform(1000, 500, 5, 1)
    assert ssp.validate_csr(_dev(ssp, A)) == 0
    bad = workloads.CSR(A.nrows, A.ncols, A.rpt.copy(), A.col.copy())
    bad.col[[3, 17, 900]] = [500, -1, 100000]
    bad.rpt[10] = bad.rpt[11] + 1
    expect = int((bad.col < 0).sum() + (bad.col >= bad.ncols).sum() +
                 (np.diff(bad.rpt) < 0).sum() + (bad.rpt[0] != 0) + (bad.rpt[-1] != bad.nnz))
    assert expect == 4
    assert ssp.validate_csr(_dev(ssp, bad)) == expect


# ------------------------------------------------------------ full size

def test_full_uniform4096(ssp):
    w = workloads.uniform4096()
    _say("full uniform4096")
    check_all(ssp, w.A, w.B, w.rate, w.seed)


def test_full_rmat20(ssp):
    w = workloads.rmat20()
    _say(f"full rmat20 nnz={w.A.nnz}")
    Ad = _dev(ssp, w.A)
    check_predict(ssp, w.A, w.A, w.rate, w.seed, Ad=Ad, Bd=Ad)
    check_reference(ssp, w.A, w.A, w.rate, w.seed, Ad=Ad, Bd=Ad)
    # exact structure: every row against the oracle's stored result (the
    # serial oracle takes many minutes), and sampled rows recomputed here
    check_exact(ssp, w.A, w.A, Ad=Ad, Bd=Ad, golden="rmat20")


def _stencil_closed_form(n):
    c = np.array([1 + min(x, 2) + min(n - 1 - x, 2) for x in range(n)])
    r = np.arange(n ** 3)
    return c[r % n] * c[(r // n) % n] * c[r // (n * n)]


def test_full_stencil128(ssp):
    w = workloads.stencil128()
    _say("full stencil128")
    Ad = _dev(ssp, w.A)
    check_predict(ssp, w.A, w.A, w.rate, w.seed, Ad=Ad, Bd=Ad)
    ex, st = ssp.exact_structure(Ad, Ad)
    torch.cuda.synchronize()
    assert np.array_equal(ex.cpu().numpy(), _stencil_closed_form(128))
    s = ssp.read_stats(st)
    assert s["out_sum"] == 634 ** 3 and s["total_flop"] == 1142 ** 3


def test_full_stencil128_times_uniform(ssp):
    w = workloads.stencil128_x_uniform()
    _say("full stencil128 x uniform")
    Ad, Bd = _dev(ssp, w.A), _dev(ssp, w.B)
    check_predict(ssp, w.A, w.B, w.rate, w.seed, Ad=Ad, Bd=Bd)
    check_exact(ssp, w.A, w.B, Ad=Ad, Bd=Bd, golden="stencil128_x_uniform")
