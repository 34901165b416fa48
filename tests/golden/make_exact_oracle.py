"""Writes exact_oracle.json: the CPU oracle's exact structure (the precise
method, Sec. I: the distinct columns of every row of C) of the full-size
products whose every row the serial oracle cannot recompute inside a GPU test:
C = A.A for the 2^20 R-MAT workload (F = 2.1e10 products) and C = A.B for the
128^3 stencil times the 2,097,152 x 65,536 uniform B.

Per product it stores Z = NNZ(C), F, and the SHA-256 digest of nnz_exact as
little-endian int64 in row order; the GPU test hashes its array the same way.
Rows are shared out over worker processes (row r to chunk r mod 64), each
calling the oracle's per-row exact count.

Only ``workloads`` (the seeded generators) and ``oracle`` are called.
Run from the repository root:  python tests/golden/make_exact_oracle.py [workers]
"""
import hashlib
import json
import os
import sys
import time
import multiprocessing

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_oracle.json")
PRODUCTS = ("rmat20", "stencil128_x_uniform")
CHUNKS = 64

_W = None


def _init(name):
    global _W
    _W = getattr(workloads, name)()


def _chunk(k):
    rows = np.arange(k, _W.A.nrows, CHUNKS, dtype=np.int32)
    nnz, rf = oracle.rows_nnz(_W.A, _W.B, rows)
    return k, nnz, rf


def one(name, workers):
    w = getattr(workloads, name)()
    M = w.A.nrows
    nnz = np.zeros(M, dtype=np.int64)
    rf = np.zeros(M, dtype=np.uint64)
    t0 = time.time()
    # (spawned workers: the generators' threads of this process do not
    # survive a fork)
    ctx = multiprocessing.get_context("spawn")
    with ctx.Pool(workers, initializer=_init, initargs=(name,)) as pool:
        for k, cn, cr in pool.imap_unordered(_chunk, range(CHUNKS)):
            nnz[k::CHUNKS] = cn
            rf[k::CHUNKS] = cr
            print(f"{name}: chunk {k} done {time.time() - t0:.0f}s", flush=True)
    return {"name": w.name, "nrows": M, "nnz_A": int(w.A.nnz), "nnz_B": int(w.B.nnz),
            "Z": int(nnz.sum()), "F": int(rf.sum(dtype=np.uint64)),
            "nnz_exact_sha256": hashlib.sha256(nnz.astype("<i8").tobytes()).hexdigest()}


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else max(1, (os.cpu_count() or 2) - 1)
    oracle.build()
    recs = {p: one(p, workers) for p in PRODUCTS}
    about = ("Oracle exact structure (every row) of full-size products: Z, F and SHA-256 of "
             "nnz_exact as little-endian int64; written by tests/golden/make_exact_oracle.py "
             "from oracle/ and workloads/ only")
    with open(OUT, "w") as f:
        json.dump({"_about": about, **recs}, f, indent=1)
        f.write("\n")
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
