"""Writes sweep_oracle.json: the CPU oracle's prediction of every case of the
625-product sweep (the workload shape of the paper's 625 pairwise products,
Sec. VI-A), for the GPU parity test of the batched and graph-captured calls.

Per case it stores the oracle's statistics (F, n_s, f*, z*, the sum of the
per-row predictions, M, flags, the sampled rows' entries of A) and SHA-256
digests of its per-row outputs, nnz_pred and row_flop, each as little-endian
int64 bytes in row order.  The arrays themselves (1.4 GB each over the sweep)
are not stored: the test hashes the GPU's arrays the same way and compares.

Only ``workloads`` (the seeded generators) and ``oracle`` are called.
Run from the repository root:  python tests/golden/make_sweep_oracle.py [workers]
"""
import hashlib
import json
import os
import sys
import time
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sweep_oracle.json")
STAT_KEYS = ("total_flop", "n_sampled", "sample_flop", "sample_nnz", "out_sum", "nrows", "flags",
             "a_sample_nnz")


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


def one(case):
    w = workloads.sweep_workload(case)
    pred, rf, st = oracle.predict(w.A, w.B, w.rate, w.seed, oracle.BERNOULLI)
    rec = {"case": list(case), "name": w.name, "nnz_A": int(w.A.nnz),
           "nnz_pred_sha256": digest(pred), "row_flop_sha256": digest(rf.astype(np.int64))}
    for k in STAT_KEYS:
        rec[k] = int(getattr(st, k))
    return rec


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else max(1, (os.cpu_count() or 2) - 1)
    oracle.build()
    cases = workloads.sweep_cases()
    # costly cases first (R-MAT, large, dense) so the pool ends evenly
    order = sorted(range(len(cases)),
                   key=lambda i: -(cases[i][1] * cases[i][2] ** 2 *
                                   (64 if cases[i][0] == "rmat" else 1)))
    t0 = time.time()
    recs = [None] * len(cases)
    with Pool(workers) as pool:
        for k, (i, rec) in enumerate(zip(order, pool.imap(one, [cases[i] for i in order]))):
            recs[i] = rec
            if k % 25 == 0:
                print(f"{k + 1}/{len(cases)} {rec['name']} {time.time() - t0:.0f}s", flush=True)
    about = ("Oracle predictions of the 625-case sweep (sizes 2^12..2^20, d 2..32, five "
             "structures, generator seeds 1..5, rate 1%, sampler seed 1000 + generator seed): "
             "statistics and SHA-256 of nnz_pred and row_flop as little-endian int64; written "
             "by tests/golden/make_sweep_oracle.py from oracle/ and workloads/ only")
    with open(OUT, "w") as f:  # one line per case
        f.write('{"_about": ' + json.dumps(about) + ',\n"cases": [\n')
        f.write(",\n".join(json.dumps(r, separators=(",", ":")) for r in recs))
        f.write("\n]}\n")
    print(f"wrote {OUT}: {len(recs)} cases in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
