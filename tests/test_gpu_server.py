"""Serving with continuous batching: every request's result equals the
per-matrix call and the CPU oracle bit for bit, alone or in a mix of
concurrent requests; batches run on several slots at once; errors come back
at submission."""
import os
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import workloads
from tests.test_gpu_parity import STAT_KEYS

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


@pytest.fixture(scope="module")
def pool(ssp):
    specs = [("uniform", 4096, 8), ("rmat", 1 << 17, 16), ("banded", 30011, 4),
             ("blockdiag", 50000, 8), ("zipf", 70001, 8), ("rmat", 1 << 15, 32),
             ("uniform", 1200, 2), ("zipf", 200_000, 4), ("blockdiag", 1 << 18, 16)]
    mats = [workloads.make(s, n, d, 20 + i) for i, (s, n, d) in enumerate(specs)]
    return mats, [ssp.DeviceCSR.from_csr(m, "cuda:0") for m in mats]


def _buffers(devs, j):
    """Output buffers of a request on matrix j.  The server's streams do not
    wait for torch's, so the caller synchronizes before handing them over
    (the fill, and any earlier use of the memory, must be done)."""
    return (torch.empty(devs[j].nrows, dtype=torch.int64, device="cuda:0"),
            torch.zeros(8, dtype=torch.int64, device="cuda:0"))


def _submit(srv, ids, devs, j, rate, seed, bufs=None):
    if bufs is None:
        bufs = _buffers(devs, j)
        torch.cuda.synchronize()
    out, st = bufs
    t = srv.submit(ids[j], ids[j], rate, seed, out, st)
    return t, j, rate, seed, out, st


def _alone(ssp, devs, j, rate, seed):
    p, _, st = ssp.predict_structure(devs[j], devs[j], rate, seed)
    return p, st


def _oracle_many(jobs):
    """oracle.predict of every (matrix, rate, seed) job, on a thread pool (the
    oracle's C calls release the interpreter lock)."""
    workers = max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as ex:
        res = list(ex.map(lambda j: oracle.predict(j[0], j[0], j[1], j[2]), jobs))
    return res


def test_server_results_equal_single_calls(ssp, pool):
    mats, devs = pool
    srv = ssp.Server(slots=3, slot_bytes=1 << 30, max_batch=16)
    ids = [srv.register(d) for d in devs]
    rng = np.random.default_rng(7)
    reqs = []
    # a burst, then a trickle: arrivals while batches run join later batches
    # (every request's buffers made ready before the first submission)
    burst = [(int(rng.integers(len(devs))), float(rng.choice([0.01, 0.05, 0.3])), 100 + i)
             for i in range(60)]
    trickle = [(int(rng.integers(len(devs))), 0.02, 300 + i) for i in range(40)]
    bufs = [_buffers(devs, j) for j, _, _ in burst + trickle]
    torch.cuda.synchronize()
    for i, (j, rate, seed) in enumerate(burst):
        reqs.append(_submit(srv, ids, devs, j, rate, seed, bufs[i]))
    for i, (j, rate, seed) in enumerate(trickle):
        time.sleep(float(rng.exponential(2e-4)))
        reqs.append(_submit(srv, ids, devs, j, rate, seed, bufs[len(burst) + i]))
    for r in reqs:
        srv.wait(r[0], 120.0)
    info = srv.info()
    _say(f"server info {info}")
    assert info["submitted"] == info["completed"] == len(reqs)
    assert info["max_batch_seen"] > 1 and info["batches"] < len(reqs)
    assert 0 < info["latency_p50_ms"] <= info["latency_p99_ms"] <= info["latency_max_ms"]
    for t, j, rate, seed, out, st in reqs:
        p, s = _alone(ssp, devs, j, rate, seed)
        torch.cuda.synchronize()
        assert torch.equal(out, p), f"ticket {t}: nnz_pred differs from the single call"
        assert torch.equal(st, s), f"ticket {t}: stats differ from the single call"
    srv.close()
    # every served result against the CPU oracle
    t0 = time.time()
    orc = _oracle_many([(mats[j], rate, seed) for _, j, rate, seed, _, _ in reqs])
    _say(f"oracle for {len(reqs)} requests in {time.time() - t0:.1f}s")
    for (t, j, rate, seed, out, st), (o_pred, _, o_st) in zip(reqs, orc):
        assert np.array_equal(out.cpu().numpy(), o_pred), f"ticket {t}: nnz_pred != oracle"
        got = ssp.read_stats(st)
        for k in STAT_KEYS:
            assert got[k] == getattr(o_st, k), f"ticket {t}: stats.{k} != oracle"


def test_server_request_alone_equals_request_in_mix(ssp, pool):
    _, devs = pool
    srv = ssp.Server(slots=3, slot_bytes=1 << 30, max_batch=2)
    ids = [srv.register(d) for d in devs]
    t, *_, out_alone, st_alone = _submit(srv, ids, devs, 1, 0.05, 42)
    srv.wait(t, 60.0)
    srv.reset_stats()
    first = [(k % len(devs), 0.03, 500 + k) for k in range(12)]
    second = [((3 * k + 1) % len(devs), 0.04, 900 + k) for k in range(12)]
    bufs = [_buffers(devs, j) for j, _, _ in first + [(1, 0, 0)] + second]
    torch.cuda.synchronize()
    mix = [_submit(srv, ids, devs, j, r, sd, bufs[i]) for i, (j, r, sd) in enumerate(first)]
    probe = _submit(srv, ids, devs, 1, 0.05, 42, bufs[len(first)])
    mix += [_submit(srv, ids, devs, j, r, sd, bufs[len(first) + 1 + i])
            for i, (j, r, sd) in enumerate(second)]
    for r in mix + [probe]:
        srv.wait(r[0], 120.0)
    info = srv.info()
    _say(f"mix info {info}")
    assert info["max_slots_busy"] >= 2, "batches never ran on two slots at once"
    assert torch.equal(probe[4], out_alone) and torch.equal(probe[5], st_alone)
    srv.close()


def test_server_errors(ssp, pool):
    _, devs = pool
    with pytest.raises(ssp.SspError):
        ssp.Server(slots=0)
    with pytest.raises(ssp.SspError):
        ssp.Server(slots=1, slot_bytes=4096)  # smaller than the shared part of a plan
    small = ssp.Server(slots=1, slot_bytes=(1 << 27) + (1 << 20), max_batch=4)
    ids = [small.register(d) for d in devs]
    out = torch.empty(devs[8].nrows, dtype=torch.int64, device="cuda:0")
    with pytest.raises(ssp.SspError) as ei:  # does not fit a slot alone
        small.submit(ids[8], ids[8], 0.5, 1, out)
    assert ei.value.status == -4
    with pytest.raises(ssp.SspError) as ei:
        small.submit(99, 0, 0.5, 1, out)
    assert ei.value.status == -1
    with pytest.raises(ssp.SspError) as ei:
        small.submit(ids[0], ids[0], 1.5, 1, out)
    assert ei.value.status == -1
    with pytest.raises(ssp.SspError):
        small.poll(123456)
    small.close()
