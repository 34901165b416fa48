"""The prediction entry point that allocates nothing
(ssp_predict_structure_noalloc, through the C ABI) equals the allocating one
(ssp_predict_structure_ex), bit for bit, outputs and statistics, on two calls
in a row (the second on a smaller input, so the fixed scratch holds the first
call's contents), and both equal the CPU oracle.  A product whose workspace
does not fit the fixed scratch is refused before anything is queued.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.test_gpu_parity import STAT_KEYS, _long_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2207_13848_amd as m
    return m


def _say(msg):
    print(msg, flush=True)


def _both(ssp, A, B, rate, seed, sampler):
    dev = "cuda:0"
    Ad = ssp.DeviceCSR.from_csr(A, dev)
    Bd = Ad if B is A else ssp.DeviceCSR.from_csr(B, dev)
    M = A.nrows
    pred, rf, st = ssp.predict_structure(Ad, Bd, rate, seed, sampler=sampler,
                                         return_row_flop=True)
    # outputs pre-filled with garbage: the call must write every element
    out = torch.full((M,), -7, dtype=torch.int64, device=dev)
    rf2 = torch.full((M,), -7, dtype=torch.int64, device=dev)
    st2 = torch.full((8,), -7, dtype=torch.int64, device=dev)
    ssp.predict_structure_noalloc(Ad, Bd, rate, seed, sampler=sampler, out=out, row_flop=rf2,
                                  stats=st2)
    # and without the row-FLOP output (its workspace array then sits in the scratch)
    out3 = torch.full((M,), -7, dtype=torch.int64, device=dev)
    st3 = torch.full((8,), -7, dtype=torch.int64, device=dev)
    ssp.predict_structure_noalloc(Ad, Bd, rate, seed, sampler=sampler, out=out3, stats=st3)
    torch.cuda.synchronize()
    ref = pred.cpu().numpy()
    assert np.array_equal(out.cpu().numpy(), ref), "nnz_pred differs from the allocating call"
    assert np.array_equal(out3.cpu().numpy(), ref), "nnz_pred (no row_flop) differs"
    assert np.array_equal(rf2.cpu().numpy(), rf.cpu().numpy()), "row_flop differs"
    s_ref = ssp.read_stats(st)
    assert ssp.read_stats(st2) == s_ref and ssp.read_stats(st3) == s_ref, "stats differ"
    mode = oracle.PAPER if sampler == "paper" else oracle.BERNOULLI
    o_pred, o_rf, o_st = oracle.predict(A, B, rate, seed, mode)
    assert np.array_equal(ref, o_pred), "nnz_pred differs from the oracle"
    assert np.array_equal(rf2.cpu().numpy(), o_rf.astype(np.int64))
    for k in STAT_KEYS:
        assert s_ref[k] == getattr(o_st, k), k
    return s_ref


def test_noalloc_equals_allocating_call_twice(ssp):
    # first: R-MAT 2^16 (hub rows split into parts, whose bitmaps sit in the
    # scratch); second, smaller (fewer rows and entries) on the same scratch:
    # long rows split into parts over B wider than one bitmap window
    W = workloads.make("rmat", 1 << 16, 16, 5)
    _say(f"noalloc call 1: rmat {W.nrows} rows, {W.nnz} entries, rate 0.05")
    s1 = _both(ssp, W, W, 0.05, 1005, "bernoulli")
    A, B = _long_rows((1 << 21) + 12345, 5, 2)
    _say(f"noalloc call 2: long rows {A.nrows}x{A.ncols} ({A.nnz} entries) . "
         f"{B.nrows}x{B.ncols}, rate 1")
    assert A.nrows < W.nrows and A.nnz < W.nnz
    s2 = _both(ssp, A, B, 1.0, 3, "bernoulli")
    assert s2["n_sampled"] == A.nrows < s1["nrows"]
    U = workloads.uniform(4096, 4096, 8, 1)
    _say("noalloc call 3: uniform 4096, paper sampler")
    _both(ssp, U, U, 0.01, 1001, "paper")


def test_noalloc_holds_the_largest_workloads(ssp):
    # 2^21 rows (the stencil's and the largest request's row count) fit the
    # fixed scratch with every part window of the allocating call
    U = workloads.uniform(1 << 21, 1 << 21, 4, 3)
    _say(f"noalloc: uniform {U.nrows} rows, d 4")
    s = _both(ssp, U, U, 0.005, 1003, "bernoulli")
    assert s["nrows"] == 1 << 21


def test_noalloc_refuses_a_product_beyond_its_scratch(ssp):
    # 5,000,000 empty rows: a valid product (every count 0) whose plan needs
    # more than the fixed 256 MiB
    M = 5_000_000
    E = workloads.CSR(M, M, np.zeros(M + 1, np.int32), np.zeros(0, np.int32), "empty5m")
    Ed = ssp.DeviceCSR.from_csr(E, "cuda:0")
    out = torch.zeros(M, dtype=torch.int64, device="cuda:0")
    st = torch.zeros(8, dtype=torch.int64, device="cuda:0")
    _say("noalloc: refusal beyond the scratch")
    with pytest.raises(ssp.SspError) as ei:
        ssp.predict_structure_noalloc(Ed, Ed, 0.01, 1, out=out, stats=st)
    assert ei.value.status == -4  # SSP_ERR_BUDGET
    assert "fixed array" in str(ei.value)
    # the allocating call handles it
    pred, _, st2 = ssp.predict_structure(Ed, Ed, 0.01, 1)
    torch.cuda.synchronize()
    assert int(pred.abs().sum()) == 0
    assert ssp.read_stats(st2)["nrows"] == M
