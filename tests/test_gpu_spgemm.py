"""Numeric product sized by the prediction: GPU path == CPU oracle, through the C ABI.

Integer parts (C's row offsets and columns, the slot layout's counts) must be
equal element by element.  Values are sums of float64 products whose order
differs (the GPU adds with atomics), so they are compared against the error
bound of any summation order: for an entry of n terms p_k, each side is
within n u sum|p_k| of the exact sum (u = 2^-53; products rounded once,
sums n - 1 times), so the two differ by at most 2 (n + 1) u sum|p_k|.  With
small-integer values every partial sum is exact and the values must be equal.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.csr_util import from_rows, random_csr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def ssp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2207_13848_amd as m
    return m


def _say(msg):
    print(msg, flush=True)


def _run(ssp, A, B, av, bv, cap, margin, Ad=None, Bd=None, capacity=None, spill=0):
    Ad = Ad if Ad is not None else ssp.DeviceCSR.from_csr(A, "cuda:0")
    Bd = Bd if Bd is not None else (Ad if B is A else ssp.DeviceCSR.from_csr(B, "cuda:0"))
    tav = torch.from_numpy(np.ascontiguousarray(av)).to("cuda:0")
    tbv = tav if bv is av else torch.from_numpy(np.ascontiguousarray(bv)).to("cuda:0")
    tcap = cap if isinstance(cap, torch.Tensor) else torch.from_numpy(
        np.ascontiguousarray(cap, dtype=np.int64)).to("cuda:0")
    rpt, col, val, info = ssp.spgemm(Ad, tav, Bd, tbv, tcap, margin_pct=margin, spill_pct=spill,
                                     capacity=capacity)
    torch.cuda.synchronize()
    return rpt.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy(), info, tcap.cpu().numpy()


def check(ssp, A, B, av, bv, cap, margin, exact_values, what, held=None, **kw):
    """Runs the product and compares it with the oracle.  ``held``: every
    overflowing row must end in the overflow area (True), none (False), or
    either (None: an area that may run short)."""
    _say(f"spgemm {what}: M={A.nrows} K={A.ncols} N={B.ncols} margin={margin} "
         f"spill={kw.get('spill', 0)}")
    rpt, col, val, info, cap_np = _run(ssp, A, B, av, bv, cap, margin, **kw)
    orpt, ocol, oval, oabs, oterms = oracle.spgemm(A, av, B, bv)
    assert np.array_equal(rpt, orpt), f"{what}: C_rpt"
    assert np.array_equal(col, ocol), f"{what}: C_col"
    if exact_values:
        assert np.array_equal(val, oval), f"{what}: C_val (integer values)"
    else:
        bound = 2.0 * (oterms.astype(np.float64) + 1.0) * U * oabs * (1.0 + 1e-9)
        bad = np.nonzero(np.abs(val - oval) > bound)[0]
        assert bad.size == 0, f"{what}: C_val beyond the bound at {bad[:5]}"
    lay = oracle.spgemm_layout(cap_np, margin, np.diff(orpt), B.ncols)
    _, F = oracle.row_flop(A, B)
    for k, v in lay.items():
        assert info[k] == v, f"{what}: info.{k} gpu={info[k]} oracle={v}"
    assert info["total_flop"] == F, f"{what}: F"
    assert 0 <= info["spill_rows"] <= info["overflow_rows"], what
    assert 0 <= info["spill_nnz"] <= info["overflow_nnz"], what
    if kw.get("spill", 0) == 0:
        assert info["spill_rows"] == info["spill_nnz"] == info["spill_bytes"] == 0, what
    if held is not None:
        # an area large enough: every overflowing row of at most 256 products
        # or (B's rows sorted) more than 2048 ends in it, a row in between may
        # (when it completes within half its table); a row of more than 2048
        # products keeps its first s_i entries in its slot, a shorter row none
        cnt = np.diff(orpt)
        rf = np.asarray(oracle.row_flop(A, B)[0])
        slot = _slots(cap_np, margin, B.ncols)
        over = cnt > slot
        sure = over & ((rf <= 256) | (rf > 2048))
        maybe = over & ~sure
        kept = np.where(rf > 2048, cnt - slot, cnt)
        if held:
            assert sure.sum() <= info["spill_rows"] <= sure.sum() + maybe.sum(), what
            assert kept[sure].sum() <= info["spill_nnz"] <= kept[sure].sum() + kept[maybe].sum(), what
            if not maybe.any():
                assert info["spill_rows"] == lay["overflow_rows"], what
        else:
            assert info["spill_rows"] == 0, what
    return info


def _slots(cap, margin, N):
    c = np.clip(np.asarray(cap, dtype=np.int64), 0, N)
    return np.minimum(N, c + (c * margin + 99) // 100)


def _values(M, seed, kind):
    return workloads.values(M.nnz, seed, kind)


CASES = [
    ("uniform3000_d8", lambda: workloads.uniform(3000, 3000, 8, 1)),
    ("zipf4096_d6", lambda: workloads.zipf(4096, 6, 2)),
    ("banded2500_d12", lambda: workloads.banded(2500, 12, 3)),
    ("rmat12_d8", lambda: workloads.rmat(1 << 12, 8, 4)),
    ("blockdiag3000_d16", lambda: workloads.blockdiag(3000, 16, 5)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("kind", ["int", "uniform"])
def test_spgemm_predicted_capacity(ssp, name, make, kind):
    A = make()
    av = _values(A, 7, kind)
    Ad = ssp.DeviceCSR.from_csr(A, "cuda:0")
    pred, _ = ssp.predict_structure(Ad, Ad, 0.02, 11)[:2]
    for margin in (0, 10):
        check(ssp, A, A, av, av, pred, margin, kind == "int", f"{name}/{kind}/pred", Ad=Ad, Bd=Ad)


def test_spgemm_capacity_kinds(ssp):
    A = workloads.zipf(3000, 8, 9)
    av = _values(A, 3, "int")
    counts, _ = oracle.exact(A, A)
    rf, _ = oracle.row_flop(A, A)
    Ad = ssp.DeviceCSR.from_csr(A, "cuda:0")
    # the precise structure: nothing overflows
    info = check(ssp, A, A, av, av, counts, 0, True, "exact caps", Ad=Ad, Bd=Ad)
    assert info["overflow_rows"] == 0
    # the upper bound
    info = check(ssp, A, A, av, av, np.asarray(rf, dtype=np.int64), 0, True, "flop caps", Ad=Ad, Bd=Ad)
    assert info["overflow_rows"] == 0
    # no capacity: every row goes through the fallback pass
    info = check(ssp, A, A, av, av, np.zeros(A.nrows, dtype=np.int64), 0, True, "zero caps",
                 Ad=Ad, Bd=Ad)
    assert info["overflow_nnz"] == info["nnz"]
    # half the exact counts, negative and huge capacities, a margin
    rng = np.random.default_rng(1)
    caps = counts // 2
    caps[rng.random(A.nrows) < 0.1] = -5
    caps[rng.random(A.nrows) < 0.1] = 1 << 40
    check(ssp, A, A, av, av, caps, 37, True, "mixed caps", Ad=Ad, Bd=Ad)


def test_spgemm_long_rows_dense_path(ssp):
    # rows of about 4096 products: every row in the dense accumulators;
    # N above 2^16 and a rectangular B
    A = workloads.uniform(1500, 2000, 64, 2)
    B = workloads.uniform(2000, 70000, 64, 3)
    av, bv = _values(A, 1, "uniform"), _values(B, 2, "uniform")
    counts, _ = oracle.exact(A, B)
    check(ssp, A, B, av, bv, counts, 0, False, "dense exact caps")
    check(ssp, A, B, av, bv, counts - 3, 0, False, "dense overflow")
    avi, bvi = _values(A, 1, "int"), _values(B, 2, "int")
    check(ssp, A, B, avi, bvi, counts // 3, 5, True, "dense int")


def test_spgemm_mixed_bins_rmat(ssp):
    # power-law rows: every bin, the dense path included, with under-predicted rows
    A = workloads.rmat(1 << 13, 12, 6)
    av = _values(A, 4, "uniform")
    Ad = ssp.DeviceCSR.from_csr(A, "cuda:0")
    rf, _ = oracle.row_flop(A, A)
    assert max(rf) > 2048 and min(r for r in rf if r) <= 128
    pred, _ = ssp.predict_structure(Ad, Ad, 0.01, 3)[:2]
    check(ssp, A, A, av, av, pred, 0, False, "rmat13 pred", Ad=Ad, Bd=Ad)


def test_spgemm_duplicates_unsorted(ssp):
    rng = np.random.default_rng(3)
    A = random_csr(rng, 700, 300, 0.04, dup_prob=0.3)
    B = random_csr(rng, 300, 900, 0.05, dup_prob=0.3)
    av, bv = _values(A, 5, "int"), _values(B, 6, "int")
    counts, _ = oracle.exact(A, B)
    check(ssp, A, B, av, bv, counts - 1, 0, True, "duplicates")


def test_spgemm_edges(ssp):
    # empty rows, rows naming only empty B rows, an empty A, no entries at all
    B = from_rows([[0, 3], [], [1], [2, 3, 4]], 5)
    bv = np.arange(1.0, B.nnz + 1.0)
    A = from_rows([[], [1], [0, 1, 2], [3], [], [1, 1]], 4)
    av = np.array([1.0, 2.0, -1.0, 3.0, 4.0, 5.0, 6.0])[: A.nnz]
    check(ssp, A, B, av, bv, np.array([0, 0, 1, 9, 0, 0]), 0, True, "small")
    A0 = from_rows([], 4)
    check(ssp, A0, B, np.zeros(0), bv, np.zeros(0, dtype=np.int64), 0, True, "no rows")
    Ae = from_rows([[], [], []], 4)
    check(ssp, Ae, B, np.zeros(0), bv, np.zeros(3, dtype=np.int64), 0, True, "no entries")
    Bz = from_rows([[], [], [], []], 0)
    check(ssp, A, Bz, av, np.zeros(0), np.ones(A.nrows, dtype=np.int64), 0, True, "N = 0")


def test_spgemm_repeated_calls_and_capacity_error(ssp):
    # a second call reuses the handle's buffers (accumulators zero again)
    A = workloads.uniform(800, 800, 48, 8)
    av = _values(A, 2, "int")
    counts, _ = oracle.exact(A, A)
    Ad = ssp.DeviceCSR.from_csr(A, "cuda:0")
    for r in range(3):
        check(ssp, A, A, av, av, counts // (r + 1), 0, True, f"repeat {r}", Ad=Ad, Bd=Ad)
    with pytest.raises(ssp.SspError):
        _run(ssp, A, A, av, av, counts, 0, Ad=Ad, Bd=Ad, capacity=int(counts.sum()) - 1)
    # and works again afterwards
    check(ssp, A, A, av, av, counts, 0, True, "after error", Ad=Ad, Bd=Ad)


def _shuffled_rows(M, vals, seed):
    """The same matrix with every row's entries (and values) in random order."""
    rng = np.random.default_rng(seed)
    col, v = M.col.copy(), vals.copy()
    for i in range(M.nrows):
        a, b = int(M.rpt[i]), int(M.rpt[i + 1])
        p = rng.permutation(b - a)
        col[a:b], v[a:b] = col[a:b][p], v[a:b][p]
    return workloads.CSR(M.nrows, M.ncols, M.rpt, col, M.name + "_shuffled"), v


def _doubled_entries(M, vals):
    """Every entry stored twice, next to itself (rows stay non-decreasing)."""
    col = np.repeat(M.col, 2)
    v = np.repeat(vals, 2) * 0.5
    return workloads.CSR(M.nrows, M.ncols, (M.rpt * 2).astype(np.int32), col, M.name + "_x2"), v


def test_spgemm_long_rows_unsorted_b(ssp):
    # rows of B not sorted: the long rows take the global-accumulator kernel
    A = workloads.uniform(600, 2000, 64, 5)
    B, bv = _shuffled_rows(workloads.uniform(2000, 30000, 64, 6), _values(
        workloads.uniform(2000, 30000, 64, 6), 2, "int"), 3)
    av = _values(A, 1, "int")
    counts, _ = oracle.exact(A, B)
    check(ssp, A, B, av, bv, counts, 0, True, "dense, unsorted B")
    check(ssp, A, B, av, bv, counts - 5, 0, True, "dense, unsorted B, overflow")


def test_spgemm_long_rows_repeated_columns(ssp):
    # sorted rows of B with every column twice: the column-window kernel
    A = workloads.uniform(500, 1500, 48, 7)
    B0 = workloads.uniform(1500, 50000, 40, 8)
    B, bv = _doubled_entries(B0, _values(B0, 3, "int"))
    av = _values(A, 4, "int")
    counts, _ = oracle.exact(A, B)
    check(ssp, A, B, av, bv, counts, 0, True, "dense, repeated columns")
    check(ssp, A, B, av, bv, counts // 2, 0, True, "dense, repeated columns, overflow")


def test_spgemm_large_tables_team_kernels(ssp):
    # rows of 1024..2048 products with over a thousand distinct columns: tables of
    # 4096 slots (the 512-thread kernel) and of 2048 (the 256-thread kernel)
    A = workloads.uniform(3000, 3000, 40, 11)
    av = _values(A, 6, "int")
    counts, _ = oracle.exact(A, A)
    assert counts.min() > 700
    check(ssp, A, A, av, av, counts, 0, True, "bin 3, 4096-slot tables")
    B = workloads.uniform(3000, 3000, 20, 12)
    bv = _values(B, 7, "int")
    counts2, _ = oracle.exact(A, B)
    check(ssp, A, B, av, bv, counts2, 0, True, "bin 2, 2048-slot tables")
    check(ssp, A, B, av, bv, counts2 // 2, 0, True, "bin 2, overflow")


def test_spgemm_long_rows_unsorted_wide_b(ssp):
    # unsorted B wider than 2^19 columns: the accumulators' bitmap in global memory
    A = workloads.uniform(300, 2000, 64, 13)
    B0 = workloads.uniform(2000, 600000, 64, 14)
    B, bv = _shuffled_rows(B0, _values(B0, 8, "int"), 5)
    av = _values(A, 9, "int")
    counts, _ = oracle.exact(A, B)
    check(ssp, A, B, av, bv, counts, 0, True, "dense, unsorted B, N = 600000")
    check(ssp, A, B, av, bv, counts - 7, 0, True, "dense, unsorted B, N = 600000, overflow")


def test_spgemm_window_search_entry_counts(ssp):
    # long rows of 1 to 2100 A entries over sorted B rows of up to 12,000
    # entries spanning seven column windows: every group size of the window
    # search (64 lanes per A entry down to one thread per entry), rows whose
    # entries fill several chunks of the workgroup (their cursors in global
    # scratch), rows of few products per window, B rows with every column
    # twice, and short rows beside them
    rng = np.random.default_rng(31)
    K, N = 4000, 110000
    longb = rng.random(K) < 0.1
    blen = np.where(longb, rng.integers(3000, 6000, K), rng.integers(0, 60, K))
    brows = []
    for k in range(K):
        r = np.sort(rng.choice(N, size=int(blen[k]), replace=False))
        if longb[k] and k % 4 == 0:
            r = np.repeat(r, 2)
        brows.append(r)
    B = from_rows(brows, N)
    long_ids, short_ids = np.nonzero(longb)[0], np.nonzero(~longb)[0]
    arows = []
    for n in (1, 2, 3, 16, 17, 33, 64, 100, 257, 300, 513, 600, 1024, 1025, 1100, 2049, 2100):
        first = rng.choice(long_ids, size=min(n, 3), replace=False)
        rest = rng.choice(K, size=n - len(first), replace=False) if n > 3 else []
        arows.append(np.concatenate([first, np.asarray(rest, dtype=np.int64)]))
    for nl, ns in ((1, 7), (2, 14), (1, 30), (1, 63), (3, 61)):
        # long rows with few products per window
        arows.append(np.concatenate([rng.choice(long_ids, size=nl, replace=False),
                                     rng.choice(short_ids, size=ns, replace=False)]))
    for _ in range(40):  # short rows (the hash bins)
        arows.append(rng.choice(short_ids, size=int(rng.integers(0, 8)), replace=False))
    rng.shuffle(arows)
    A = from_rows([np.sort(r) for r in arows], K)
    av, bv = _values(A, 12, "int"), _values(B, 13, "int")
    counts, _ = oracle.exact(A, B)
    rf = np.asarray(oracle.row_flop(A, B)[0])
    assert (rf > 2048).sum() >= 22
    check(ssp, A, B, av, bv, counts, 0, True, "window search, exact caps")
    check(ssp, A, B, av, bv, counts - 1, 0, True, "window search, fallback pass")
    check(ssp, A, B, av, bv, counts // 3, 0, True, "window search, area 300%", spill=300,
          held=True)


# ------------------------------------------------ the overflow area


def test_spgemm_overflow_area_holds_every_row(ssp):
    # power-law rows in every bin, under-predicted: with a large area no row is recomputed
    A = workloads.rmat(1 << 13, 12, 6)
    av = _values(A, 4, "uniform")
    Ad = ssp.DeviceCSR.from_csr(A, "cuda:0")
    pred, _ = ssp.predict_structure(Ad, Ad, 0.01, 3)[:2]
    info = check(ssp, A, A, av, av, pred, 0, False, "rmat13 pred, area 400%", Ad=Ad, Bd=Ad,
                 spill=400, held=True)
    assert info["overflow_rows"] > 0 and info["spill_bytes"] > 0
    avi = _values(A, 4, "int")
    check(ssp, A, A, avi, avi, pred, 10, True, "rmat13 pred +10%, area 400%", Ad=Ad, Bd=Ad,
          spill=400, held=True)


def test_spgemm_overflow_area_runs_short(ssp):
    # an area too small for every overflowing row: the rest are recomputed
    A = workloads.rmat(1 << 13, 12, 6)
    av = _values(A, 4, "int")
    Ad = ssp.DeviceCSR.from_csr(A, "cuda:0")
    pred, _ = ssp.predict_structure(Ad, Ad, 0.01, 3)[:2]
    for pct in (1, 5, 20):
        info = check(ssp, A, A, av, av, pred, 0, True, f"rmat13 pred, area {pct}%", Ad=Ad,
                     Bd=Ad, spill=pct)
        if pct == 1:
            assert info["spill_rows"] < info["overflow_rows"]


def test_spgemm_overflow_area_long_rows_across_windows(ssp):
    # rows of about 4096 products over 70,000 columns (five column windows):
    # the entries past the slot span windows; sorted B with repeated columns too
    A = workloads.uniform(1500, 2000, 64, 2)
    B = workloads.uniform(2000, 70000, 64, 3)
    av, bv = _values(A, 1, "int"), _values(B, 2, "int")
    counts, _ = oracle.exact(A, B)
    check(ssp, A, B, av, bv, counts // 3, 0, True, "dense, area 300%", spill=300, held=True)
    check(ssp, A, B, av, bv, counts - 1, 0, True, "dense, one entry over", spill=50, held=True)
    check(ssp, A, B, av, bv, np.zeros(A.nrows, dtype=np.int64), 0, True,
          "dense, zero caps (no slots, so no area)", spill=300, held=False)
    B0 = workloads.uniform(1500, 50000, 40, 8)
    B2, bv2 = _doubled_entries(B0, _values(B0, 3, "int"))
    A2 = workloads.uniform(500, 1500, 48, 7)
    av2 = _values(A2, 4, "int")
    c2, _ = oracle.exact(A2, B2)
    check(ssp, A2, B2, av2, bv2, c2 // 2, 0, True, "dense, repeated columns, area", spill=200,
          held=True)


def test_spgemm_overflow_area_chunks(ssp):
    # more entries past the slots than one chunk of the area per workgroup:
    # a row's run breaks where its workgroup takes the next chunk
    A = workloads.uniform(20000, 2000, 64, 21)
    B = workloads.uniform(2000, 40000, 64, 22)
    av, bv = _values(A, 5, "int"), _values(B, 6, "int")
    counts, _ = oracle.exact(A, B)
    info = check(ssp, A, B, av, bv, counts // 4, 0, True, "dense, area in many chunks",
                 spill=400, held=True)
    assert info["spill_nnz"] > 256 * (1 << 16)


def test_spgemm_overflow_area_unsorted_b(ssp):
    # unsorted B: the long rows' kernel keeps no overflow, the short rows do
    A = workloads.uniform(600, 2000, 64, 5)
    Bs = workloads.uniform(2000, 30000, 64, 6)
    B, bv = _shuffled_rows(Bs, _values(Bs, 2, "int"), 3)
    av = _values(A, 1, "int")
    counts, _ = oracle.exact(A, B)
    check(ssp, A, B, av, bv, counts - 5, 0, True, "dense, unsorted B, area", spill=300,
          held=False)
    Z = workloads.zipf(3000, 8, 9)
    zv = _values(Z, 3, "int")
    zc, _ = oracle.exact(Z, Z)
    Zs, zsv = _shuffled_rows(Z, zv, 4)
    check(ssp, Zs, Zs, zsv, zsv, zc // 2, 0, True, "zipf, unsorted, area", spill=300)


def test_spgemm_overflow_area_repeated_calls(ssp):
    # the area's counters and row states start afresh on every call; a
    # smaller product after a larger one
    A = workloads.rmat(1 << 13, 12, 6)
    av = _values(A, 4, "int")
    counts, _ = oracle.exact(A, A)
    Ad = ssp.DeviceCSR.from_csr(A, "cuda:0")
    check(ssp, A, A, av, av, counts // 2, 0, True, "rmat13 half caps, area", Ad=Ad, Bd=Ad,
          spill=200, held=True)
    check(ssp, A, A, av, av, counts, 0, True, "rmat13 exact caps, area", Ad=Ad, Bd=Ad,
          spill=200, held=True)
    S = workloads.uniform(900, 900, 10, 3)
    sv = _values(S, 5, "int")
    sc, _ = oracle.exact(S, S)
    check(ssp, S, S, sv, sv, sc // 2, 0, True, "uniform900 half caps, area", spill=300,
          held=True)
    check(ssp, A, A, av, av, counts // 2, 0, True, "rmat13 half caps, no area", Ad=Ad, Bd=Ad)
