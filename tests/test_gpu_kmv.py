"""The sketch estimator of related work (Sec. III): GPU == CPU oracle, through the C ABI.

Every result is an integer (rows and columns kept, products of C', the k-th
smallest distinct 53-bit hash) or a float64 computed from them in the same
order on both sides, so all must be equal; the count of distinct hashes is
compared when the sketch is exact (fewer than k values).
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.csr_util import random_csr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2207_13848_amd as m
    return m


def check(ssp, A, B, rate, k, seed, what):
    print(f"kmv {what}: M={A.nrows} N={B.ncols} rate={rate} k={k} seed={seed}", flush=True)
    Ad = ssp.DeviceCSR.from_csr(A, "cuda:0")
    Bd = Ad if B is A else ssp.DeviceCSR.from_csr(B, "cuda:0")
    g = ssp.kmv_estimate(Ad, Bd, rate, k, seed)
    o = oracle.kmv(A, B, rate, k, seed)
    for key in ("rows_kept", "cols_kept", "products", "kth_hash", "k", "nnz_sample",
                "nnz_estimate"):
        assert g[key] == o[key], f"{what}: {key} gpu={g[key]} oracle={o[key]}"
    if o["distinct"] < k:
        assert g["distinct_kept"] == o["distinct"], f"{what}: distinct"
    else:
        assert k <= g["distinct_kept"] <= o["distinct"]
    return g, o


CASES = [
    ("uniform3000_d8", lambda: workloads.uniform(3000, 3000, 8, 1), 1.0, 256),
    ("zipf4096_d6", lambda: workloads.zipf(4096, 6, 2), 0.3, 64),
    ("rmat12_d8", lambda: workloads.rmat(1 << 12, 8, 4), 0.1, 1024),
    ("stencil16", lambda: workloads.stencil27(16), 1.0, 4096),
    ("banded20000_d12", lambda: workloads.banded(20000, 12, 3), 0.1, 512),
]


@pytest.mark.parametrize("name,make,rate,k", CASES, ids=[c[0] for c in CASES])
def test_kmv_parity(ssp, name, make, rate, k):
    A = make()
    for seed in (1, 77):
        check(ssp, A, A, rate, k, seed, name)


def test_kmv_exact_mode_and_edges(ssp):
    A = workloads.uniform(500, 400, 3, 2)
    B = workloads.uniform(400, 900, 2, 3)
    g, o = check(ssp, A, B, 1.0, 4096, 5, "fewer than k values (exact)")
    _, st = oracle.exact(A, B)
    assert g["nnz_estimate"] == float(st.out_sum)
    check(ssp, A, B, 0.0, 16, 5, "nothing kept")
    rng = np.random.default_rng(2)
    C = random_csr(rng, 300, 200, 0.05, dup_prob=0.3)
    D = random_csr(rng, 200, 250, 0.05, dup_prob=0.3)
    check(ssp, C, D, 0.5, 8, 9, "duplicates, unsorted rows")
    check(ssp, C, D, 0.5, 1, 9, "k = 1")


def test_kmv_rmat18_bench_config(ssp):
    # the configuration the benchmark reports: R-MAT 2^18 d 16, p = 1/10, k = 1024
    A = workloads.rmat(1 << 18, 16, 1)
    check(ssp, A, A, 0.1, 1024, 1001, "rmat18")
