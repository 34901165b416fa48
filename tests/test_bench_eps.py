"""The benchmark's accuracy arithmetic (eps1, epsf, eps2, eps2_alloc of
Sec. VI-A, computed in bench.py from a prediction's integer statistics and the
exact total Z) equals the oracle's exact rationals, rounded once, on oracle
runs over the sweep's five structures and on hand-made degenerate statistics.
CPU only."""
import os
import sys
from dataclasses import asdict

import pytest

import oracle
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _same(got, want):
    if want is None:
        return got is None
    return got == float(want)  # the exact rational rounded once to a double


@pytest.mark.parametrize("structure", workloads.STRUCTURES)
def test_bench_eps_equal_oracle_rationals(structure):
    for n, d, g in ((4096, 8, 1), (5003, 3, 2), (20000, 16, 3)):
        A = workloads.make(structure, n, d, g)
        for rate, seed in ((0.01, 1001), (0.05, 7), (1.0, 3)):
            _, _, st = oracle.predict(A, A, rate, seed)
            _, ex = oracle.exact(A, A)
            got = bench.eps_from_stats(asdict(st), ex.out_sum)
            want = oracle.relative_errors(st, ex.out_sum)
            for k in ("eps1", "epsf", "eps2", "eps2_alloc"):
                assert _same(got[k], want[k]), (structure, n, rate, k, got[k], want[k])
            if rate == 1.0:  # the whole matrix sampled: every estimate exact
                assert got["eps1"] == got["epsf"] == got["eps2"] == 0.0


def test_bench_eps_degenerate_statistics():
    base = dict(total_flop=100, n_sampled=0, sample_flop=0, sample_nnz=0, out_sum=100,
                nrows=10, flags=1, a_sample_nnz=0)
    e = bench.eps_from_stats(base, 40)  # empty sample: no estimate
    assert e["eps1"] is None and e["epsf"] is None and e["eps2"] is None
    assert e["eps2_alloc"] == 1.5
    e = bench.eps_from_stats(dict(base, n_sampled=3, sample_flop=30, sample_nnz=12), 0)
    assert e["eps1"] is None and e["eps2"] is None and e["eps2_alloc"] is None
    assert e["epsf"] == 0.0  # F* = 30 * 10 / 3 = 100 = F
    # a case whose error needs more than 53 bits to state before the division
    big = dict(total_flop=2**62 + 1, n_sampled=3, sample_flop=2**61 + 7, sample_nnz=2**60 + 3,
               out_sum=2**61, nrows=2**31 - 1, flags=0, a_sample_nnz=5)
    Z = 2**61 + 12345
    got = bench.eps_from_stats(big, Z)
    st = oracle.Stats(**big)
    want = oracle.relative_errors(st, Z)
    for k in ("eps1", "epsf", "eps2", "eps2_alloc"):
        assert _same(got[k], want[k]), k


def test_summarise_eps_mean_and_worst():
    recs = [("a", {"eps1": 0.5, "epsf": 0.1, "eps2": -0.2, "eps2_alloc": -0.1}),
            ("b", {"eps1": -0.1, "epsf": 0.0, "eps2": -0.1, "eps2_alloc": 0.0}),
            ("b", {"eps1": None, "epsf": None, "eps2": None, "eps2_alloc": 0.3})]
    s = bench.summarise_eps(recs)
    assert s["cases"] == 2 and s["excluded"] == 1
    assert s["mean_abs_eps1"] == pytest.approx(0.3) and s["worst_abs_eps1"] == 0.5
    assert s["mean_abs_eps2"] == pytest.approx(0.15) and s["worst_abs_eps2"] == 0.2
    assert s["frac_abs_eps2_lt_abs_eps1"] == 0.5
    assert s["by_structure"]["b"]["mean_abs_eps2"] == pytest.approx(0.1)
