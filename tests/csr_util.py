"""Small CSR helpers for the tests (no part of the method)."""
import numpy as np

from workloads import CSR


def from_rows(rows, ncols, name="rows"):
    lens = [len(r) for r in rows]
    rpt = np.zeros(len(rows) + 1, dtype=np.int32)
    rpt[1:] = np.cumsum(lens)
    col = np.array([c for r in rows for c in r], dtype=np.int32)
    return CSR(len(rows), ncols, rpt, col, name)


def random_csr(rng, nrows, ncols, density, dup_prob=0.0, shuffle=True):
    """Random structure; optional duplicate entries and unsorted rows."""
    rows = []
    for _ in range(nrows):
        r = [int(c) for c in np.nonzero(rng.random(ncols) < density)[0]]
        if dup_prob > 0 and r:
            extra = [c for c in r if rng.random() < dup_prob]
            r = r + extra
        if shuffle:
            rng.shuffle(r)
        rows.append(r)
    return from_rows(rows, ncols)


def to_count_dense(M):
    """Dense integer matrix whose (i, j) entry counts stored entries (i, j)."""
    D = np.zeros((M.nrows, M.ncols), dtype=np.int64)
    for i in range(M.nrows):
        for j in range(M.rpt[i], M.rpt[i + 1]):
            D[i, M.col[j]] += 1
    return D
