"""The whole 625-case sweep (the workload shape of the paper's 625 products,
Sec. VI-A: sizes 2^12..2^20, d 2..32, five structures, five seeds, 1%
sampling) predicted as ONE batched call and as one launch of a captured batch
graph, every case compared with the CPU oracle.

The oracle's per-row outputs over the sweep (174.6 M rows each for nnz_pred
and row_flop) are stored as SHA-256 digests of their little-endian int64
bytes, beside its statistics (tests/golden/sweep_oracle.json, written by
tests/golden/make_sweep_oracle.py, which calls only the oracle and the seeded
generators).  The GPU arrays are hashed the same way: equal digests mean equal
arrays, element by element.
"""
import hashlib
import json
import os
import time

import numpy as np
import pytest

import workloads
from tests.test_gpu_parity import STAT_KEYS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "sweep_oracle.json")


@pytest.fixture(scope="module")
def ssp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2207_13848_amd as m
    return m


def _say(msg):
    print(msg, flush=True)


def _digest(t) -> str:
    return hashlib.sha256(np.ascontiguousarray(t.cpu().numpy(), dtype="<i8").tobytes()).hexdigest()


@pytest.fixture(scope="module")
def sweep(ssp):
    with open(GOLD) as f:
        gold = json.load(f)["cases"]
    params = workloads.sweep_cases()
    assert len(params) == len(gold) == 625
    t0 = time.time()
    devs = []
    for p, g in zip(params, gold):
        assert list(p) == g["case"], (p, g["case"])
        w = workloads.sweep_workload(p)
        assert w.A.nnz == g["nnz_A"], w.name
        devs.append(ssp.DeviceCSR.from_csr(w.A, "cuda:0"))
    _say(f"sweep: 625 cases generated and uploaded in {time.time() - t0:.1f}s")
    return params, gold, devs


def _fresh_cases(ssp, params, devs):
    cases = [ssp.Case(A, A, p[4], p[5], return_row_flop=True) for p, A in zip(params, devs)]
    for c in cases:  # garbage in the outputs: every element must be written
        c.pred.fill_(-3)
        c.row_flop.fill_(-3)
        c.stats.fill_(-3)
    return cases


def _check(ssp, cases, gold, what):
    torch.cuda.synchronize()
    bad = []
    for c, g in zip(cases, gold):
        st = ssp.read_stats(c.stats)
        for k in STAT_KEYS:
            if st[k] != g[k]:
                bad.append(f"{g['name']}: stats.{k} gpu={st[k]} oracle={g[k]}")
        if _digest(c.pred) != g["nnz_pred_sha256"]:
            bad.append(f"{g['name']}: nnz_pred differs from the oracle")
        if _digest(c.row_flop) != g["row_flop_sha256"]:
            bad.append(f"{g['name']}: row_flop differs from the oracle")
    assert not bad, f"{what}: {len(bad)} mismatches, first: " + "; ".join(bad[:5])


def test_sweep_one_batch_call_equals_oracle(ssp, sweep):
    params, gold, devs = sweep
    cases = _fresh_cases(ssp, params, devs)
    _say("sweep: one ssp_predict_batch call of 625 cases")
    ssp.predict_batch(cases)
    _check(ssp, cases, gold, "batch")


def test_sweep_graph_launches_equal_oracle(ssp, sweep):
    params, gold, devs = sweep
    cases = _fresh_cases(ssp, params, devs)
    _say("sweep: batch graph of 625 cases, two launches")
    g = ssp.BatchGraph(cases)
    try:
        g.launch()
        _check(ssp, cases, gold, "graph launch 1")
        for c in cases:
            c.pred.fill_(-5)
            c.row_flop.fill_(-5)
            c.stats.fill_(-5)
        g.launch()
        _check(ssp, cases, gold, "graph launch 2")
    finally:
        g.close()
