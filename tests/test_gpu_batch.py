"""Batched prediction: every case of one ssp_predict_batch call (and of every
replay of a captured batch graph) equals the per-matrix call and the CPU
oracle, bit for bit, outputs and statistics.

The batches mix cases of uneven size and kind: the five sweep generators,
A.B with B != A, B wider than one long-row bitmap window, rows long enough to
be split into parts, an empty matrix, both samplers, with and without the
row-FLOP output and caller statistics.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.csr_util import random_csr
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


def _mixed_inputs(n_extra=0):
    """(A, B, rate, seed, sampler, want_rf) tuples of uneven size and kind."""
    out = []
    for i, (s, n, d) in enumerate([("uniform", 4096, 8), ("rmat", 16384, 16), ("banded", 5003, 4),
                                   ("blockdiag", 20000, 8), ("zipf", 70001, 8),
                                   ("rmat", 1 << 16, 32), ("uniform", 1000, 2)]):
        A = workloads.make(s, n, d, 10 + i)
        out.append((A, A, (0.02, 0.05, 1.0)[i % 3], 500 + i, "paper" if i == 3 else "bernoulli",
                    i % 2 == 0))
    rng = np.random.default_rng(4)
    A = random_csr(rng, 120, 80, 0.1, dup_prob=0.2)
    B = random_csr(rng, 80, 90, 0.2, dup_prob=0.2)
    out.append((A, B, 0.5, 9, "bernoulli", True))                      # A.B, duplicates
    out.append((workloads.CSR(0, 7, np.zeros(1, np.int32), np.zeros(0, np.int32)),
                workloads.uniform(7, 5, 2, 1), 0.5, 1, "bernoulli", False))  # M = 0
    A, B = _long_rows(300_000, 8, 1)
    out.append((A, B, 1.0, 1, "bernoulli", True))                      # split long rows
    A, B = _long_rows((1 << 21) + 12345, 5, 2)
    out.append((A, B, 1.0, 3, "bernoulli", False))                     # several windows
    for k in range(n_extra):
        A = workloads.make(workloads.STRUCTURES[k % 5], 2000 + 977 * k, 2 + k % 7, 40 + k)
        out.append((A, A, 0.03, 77 + k, "bernoulli", k % 3 == 0))
    return out


def _cases(ssp, inputs, caller_stats=True):
    cases, dev = [], {}
    for A, B, rate, seed, sampler, want_rf in inputs:
        Ad = dev.setdefault(id(A), ssp.DeviceCSR.from_csr(A, "cuda:0"))
        Bd = dev.setdefault(id(B), ssp.DeviceCSR.from_csr(B, "cuda:0"))
        c = ssp.Case(Ad, Bd, rate, seed, sampler=sampler, return_row_flop=want_rf)
        if not caller_stats:
            c.stats = None
        cases.append(c)
    return cases


def _expect_single(ssp, cases):
    exp = []
    for c in cases:
        p, rf, st = ssp.predict_structure(c.A, c.B, c.sample_rate, c.seed, sampler=c.sampler,
                                          return_row_flop=True)
        exp.append((p, rf, st))
    torch.cuda.synchronize()
    return [(p.cpu().numpy(), rf.cpu().numpy(), ssp.read_stats(st)) for p, rf, st in exp]


def _check_against(ssp, cases, expect, what):
    for i, (c, (p, rf, st)) in enumerate(zip(cases, expect)):
        assert np.array_equal(c.pred.cpu().numpy(), p), f"{what}: case {i} nnz_pred"
        if c.row_flop is not None:
            assert np.array_equal(c.row_flop.cpu().numpy(), rf), f"{what}: case {i} row_flop"
        if c.stats is not None:
            s = ssp.read_stats(c.stats)
            for k in STAT_KEYS:
                assert s[k] == st[k], f"{what}: case {i} stats.{k} {s[k]} != {st[k]}"


def _check_oracle(inputs, expect, limit=3 * 10 ** 7):
    for (A, B, rate, seed, sampler, _), (p, rf, st) in zip(inputs, expect):
        F = int(oracle.row_flop(A, B)[1])
        if F > limit:
            continue
        mode = oracle.PAPER if sampler == "paper" else oracle.BERNOULLI
        o_pred, o_rf, o_st = oracle.predict(A, B, rate, seed, mode)
        assert np.array_equal(p, o_pred) and np.array_equal(rf, o_rf.astype(np.int64))
        for k in STAT_KEYS:
            assert st[k] == getattr(o_st, k), k


def test_batch_of_few_cases_matches_single_calls(ssp):
    # at most 8 cases: the case table travels in kernel arguments
    inputs = _mixed_inputs()[:8]
    cases = _cases(ssp, inputs)
    _say(f"batch of {len(cases)}")
    ssp.predict_batch(cases)
    torch.cuda.synchronize()
    expect = _expect_single(ssp, cases)
    _check_against(ssp, cases, expect, "batch")
    _check_oracle(inputs, expect)


def test_batch_of_many_cases_matches_single_calls(ssp):
    # more than 8 cases (staged case table), library-held statistics for some
    inputs = _mixed_inputs(n_extra=25)
    cases = _cases(ssp, inputs)
    for c in cases[::4]:
        c.stats = None
    _say(f"batch of {len(cases)}")
    ssp.predict_batch(cases)
    torch.cuda.synchronize()
    expect = _expect_single(ssp, cases)
    _check_against(ssp, cases, expect, "batch")
    _check_oracle(inputs, expect)


def test_batch_is_independent_of_composition(ssp):
    # a case's result does not depend on which other cases share the batch
    inputs = _mixed_inputs(n_extra=6)
    full = _cases(ssp, inputs)
    ssp.predict_batch(full)
    sub = _cases(ssp, inputs[5:12])
    ssp.predict_batch(sub)
    rev = _cases(ssp, inputs[::-1])
    ssp.predict_batch(rev)
    torch.cuda.synchronize()
    for k, c in enumerate(sub):
        assert torch.equal(c.pred, full[5 + k].pred) and torch.equal(c.stats, full[5 + k].stats)
    for k, c in enumerate(rev):
        j = len(inputs) - 1 - k
        assert torch.equal(c.pred, full[j].pred) and torch.equal(c.stats, full[j].stats)


def test_batch_graph_replays(ssp):
    inputs = _mixed_inputs(n_extra=12)
    cases = _cases(ssp, inputs)
    g = ssp.BatchGraph(cases)
    assert g.workspace_bytes > 0
    expect = _expect_single(ssp, cases)
    _say(f"graph of {len(cases)} cases, {g.workspace_bytes} workspace bytes")
    noise = torch.randn(1 << 20, device="cuda:0")
    for rep in range(4):
        for c in cases:  # poison the outputs: every replay must rewrite them
            c.pred.fill_(-7)
            c.stats.fill_(-7)
            if c.row_flop is not None:
                c.row_flop.fill_(-7)
        g.launch()
        torch.cuda.synchronize()
        _check_against(ssp, cases, expect, f"graph replay {rep}")
        noise = noise * 1.0001 + 1.0  # eager work between replays
        ssp.predict_structure(cases[1].A, cases[1].A, 0.3, rep)
        torch.cuda.synchronize()
    g.close()


def test_batch_graph_follows_input_contents(ssp):
    # same sizes, new contents: a replay predicts the new inputs
    A = workloads.zipf(30000, 8, 2)
    Ad = ssp.DeviceCSR.from_csr(A, "cuda:0")
    case = ssp.Case(Ad, Ad, 0.05, 3, return_row_flop=True)
    g = ssp.BatchGraph([case])
    g.launch()
    torch.cuda.synchronize()
    assert np.array_equal(case.pred.cpu().numpy(), oracle.predict(A, A, 0.05, 3)[0])
    # rewrite the columns in place with another valid structure of the same shape
    rng = np.random.default_rng(3)
    new_col = np.empty_like(A.col)
    for i in range(A.nrows):
        lo, hi = A.rpt[i], A.rpt[i + 1]
        new_col[lo:hi] = np.sort(rng.choice(A.ncols, size=hi - lo, replace=False))
    Ad.col.copy_(torch.as_tensor(new_col, device="cuda:0"))
    g.launch()
    torch.cuda.synchronize()
    A2 = workloads.CSR(A.nrows, A.ncols, A.rpt, new_col)
    assert np.array_equal(case.pred.cpu().numpy(), oracle.predict(A2, A2, 0.05, 3)[0])
    g.close()


def test_batch_errors(ssp):
    A = ssp.DeviceCSR.from_csr(workloads.uniform(100, 60, 3, 1), "cuda:0")
    B = ssp.DeviceCSR.from_csr(workloads.uniform(60, 40, 3, 1), "cuda:0")
    good = ssp.Case(A, B, 0.5, 1)
    bad = ssp.Case(B, A, 0.5, 1)  # 40 != 100
    with pytest.raises(ssp.SspError) as ei:
        ssp.predict_batch([good, bad])
    assert ei.value.status == -2
    bad_rate = ssp.Case(A, B, 2.0, 1)
    with pytest.raises(ssp.SspError) as ei:
        ssp.predict_batch([bad_rate])
    assert ei.value.status == -1
    assert ssp.predict_batch([]) == []
    with pytest.raises(ValueError):
        ssp.BatchGraph([])
