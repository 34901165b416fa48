"""Sampled-compression-ratio structure prediction for SpGEMM on MI355X.

Python binding of the C ABI in ``include/ssp.h``.  Every step of the method
runs in the HIP kernels of ``libssp.so``; this module only marshals arguments.
PyTorch supplies device memory and the current stream.

    import paper_2207_13848_amd as ssp
    A = ssp.DeviceCSR.from_host(rpt, col, ncols)          # int32 CSR
    pred, row_flop, stats = ssp.predict_structure(A, A, 0.01, seed=1001)

Method: Du et al., arXiv 2207.13848 -- row FLOP (Alg. 1), row sampling of A
(Sec. IV-A), exact NNZ of the sampled rows (Alg. 2), sampled compression ratio
and per-row prediction ceil(row_flop * z* / f*) (Sec. IV-D, Eq. (4)).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _native
from ._native import (FLAG_EMPTY_SAMPLE, FLAG_SATURATED, SAMPLER_BERNOULLI, SAMPLER_PAPER,
                      SspError)

__all__ = ["DeviceCSR", "Handle", "predict_structure", "predict_structure_noalloc",
           "reference_estimate", "exact_structure",
           "validate_csr", "read_stats", "default_handle", "SspError", "FLAG_EMPTY_SAMPLE",
           "FLAG_SATURATED", "SAMPLER_BERNOULLI", "SAMPLER_PAPER", "version", "spgemm",
           "kmv_estimate"]


def version() -> str:
    return _native.load().ssp_version().decode()


@dataclass
class DeviceCSR:
    """Structure-only CSR on the GPU: rpt int32[nrows+1], col int32[nnz]."""
    rpt: torch.Tensor
    col: torch.Tensor
    ncols: int

    @property
    def nrows(self) -> int:
        return int(self.rpt.numel()) - 1

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @property
    def device(self) -> torch.device:
        return self.rpt.device

    @classmethod
    def from_host(cls, rpt, col, ncols: int, device="cuda") -> "DeviceCSR":
        r = torch.as_tensor(rpt, dtype=torch.int32).to(device).contiguous()
        c = torch.as_tensor(col, dtype=torch.int32).to(device).contiguous()
        return cls(r, c, int(ncols))

    @classmethod
    def from_csr(cls, m, device="cuda") -> "DeviceCSR":
        """From any host object with rpt, col (int32 arrays) and ncols."""
        return cls.from_host(m.rpt, m.col, m.ncols, device)

    def _c(self) -> _native.SspCsr:
        if self.rpt.dtype != torch.int32 or self.col.dtype != torch.int32:
            raise TypeError("CSR arrays must be int32")
        if not (self.rpt.is_contiguous() and self.col.is_contiguous()):
            raise ValueError("CSR arrays must be contiguous")
        return _native.SspCsr(self.nrows, self.ncols, self.nnz, self.rpt.data_ptr(),
                              self.col.data_ptr() if self.nnz else 0)


class Handle:
    """Owns the library handle (and its device workspace) for one device."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self._lib = _native.load()
        h = ctypes.c_void_p()
        st = self._lib.ssp_create(ctypes.byref(h), int(device), int(hbm_budget_bytes))
        if st != 0:
            raise SspError(st, "ssp_create")
        self.ptr = h
        self.device = int(device)

    def close(self):
        if self.ptr:
            self._lib.ssp_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def workspace_bytes(self) -> int:
        return int(self._lib.ssp_workspace_bytes(self.ptr))

    def check(self, status: int, where: str):
        if status != 0:
            detail = self._lib.ssp_last_error(self.ptr).decode(errors="replace")
            raise SspError(status, where, detail)


_handles: dict = {}


def default_handle(device=None) -> Handle:
    dev = torch.device(device if device is not None else "cuda")
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    if idx not in _handles:
        _handles[idx] = Handle(idx)
    return _handles[idx]


def _stream_ptr(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _sampler_id(sampler) -> int:
    if sampler in (SAMPLER_BERNOULLI, "bernoulli"):
        return SAMPLER_BERNOULLI
    if sampler in (SAMPLER_PAPER, "paper"):
        return SAMPLER_PAPER
    raise ValueError(f"unknown sampler {sampler!r}")


def _new_stats(device) -> torch.Tensor:
    return torch.zeros(8, dtype=torch.int64, device=device)


def read_stats(stats: torch.Tensor) -> dict:
    """Copy a device ssp_stats (int64[8] tensor) to a dict of Python ints."""
    vals = [int(v) % (1 << 64) for v in stats.cpu().tolist()]
    return dict(zip(_native.STATS_FIELDS, vals))


def predict_structure(A: DeviceCSR, B: DeviceCSR, sample_rate: float, seed: int, *,
                      sampler="bernoulli", return_row_flop: bool = False, handle=None,
                      stream=None, out=None, stats=None):
    """Predicted nnz per row of C = A.B (int64[M] on A's device).

    Returns (nnz_pred, row_flop or None, stats tensor int64[8]).  Asynchronous
    on `stream` (default: torch's current stream).
    """
    h = handle or default_handle(A.device)
    M = A.nrows
    pred = out if out is not None else torch.empty(M, dtype=torch.int64, device=A.device)
    rf = torch.empty(M, dtype=torch.int64, device=A.device) if return_row_flop else None
    st = stats if stats is not None else _new_stats(A.device)
    a, b = A._c(), B._c()
    status = h._lib.ssp_predict_structure_ex(
        h.ptr, ctypes.byref(a), ctypes.byref(b), _sampler_id(sampler), float(sample_rate),
        int(seed) % (1 << 64), pred.data_ptr() if M else 0, rf.data_ptr() if rf is not None and M
        else 0, st.data_ptr(), _stream_ptr(stream))
    h.check(status, "ssp_predict_structure")
    return pred, rf, st


def predict_structure_noalloc(A: DeviceCSR, B: DeviceCSR, sample_rate: float, seed: int, *,
                              sampler="bernoulli", handle=None, stream=None, out, row_flop=None,
                              stats):
    """predict_structure into caller-given tensors, with the library's fixed
    device scratch as its workspace (ssp_predict_structure_noalloc): nothing
    is allocated, so the call may run under graph capture.  `out` (int64[M]),
    `stats` (int64[8]) and the optional `row_flop` (int64[M]) are written."""
    h = handle or default_handle(A.device)
    M = A.nrows
    a, b = A._c(), B._c()
    status = h._lib.ssp_predict_structure_noalloc(
        h.ptr, ctypes.byref(a), ctypes.byref(b), _sampler_id(sampler), float(sample_rate),
        int(seed) % (1 << 64), out.data_ptr() if M else 0,
        row_flop.data_ptr() if row_flop is not None and M else 0, stats.data_ptr(),
        _stream_ptr(stream))
    h.check(status, "ssp_predict_structure_noalloc")
    return out, row_flop, stats


def reference_estimate(A: DeviceCSR, B: DeviceCSR, sample_rate: float, seed: int, *,
                       sampler="bernoulli", handle=None, stream=None, out=None, stats=None):
    """Reference design (Sec. IV-C, Eq. (2)) on the same sample: (nnz_ref, stats)."""
    h = handle or default_handle(A.device)
    M = A.nrows
    ref = out if out is not None else torch.empty(M, dtype=torch.int64, device=A.device)
    st = stats if stats is not None else _new_stats(A.device)
    a, b = A._c(), B._c()
    status = h._lib.ssp_reference_estimate(
        h.ptr, ctypes.byref(a), ctypes.byref(b), _sampler_id(sampler), float(sample_rate),
        int(seed) % (1 << 64), ref.data_ptr() if M else 0, st.data_ptr(), _stream_ptr(stream))
    h.check(status, "ssp_reference_estimate")
    return ref, st


def exact_structure(A: DeviceCSR, B: DeviceCSR, *, handle=None, stream=None, out=None,
                    stats=None):
    """Exact nnz per row of C = A.B (the precise method): (nnz_exact, stats)."""
    h = handle or default_handle(A.device)
    M = A.nrows
    ex = out if out is not None else torch.empty(M, dtype=torch.int64, device=A.device)
    st = stats if stats is not None else _new_stats(A.device)
    a, b = A._c(), B._c()
    status = h._lib.ssp_exact_structure(h.ptr, ctypes.byref(a), ctypes.byref(b),
                                        ex.data_ptr() if M else 0, st.data_ptr(),
                                        _stream_ptr(stream))
    h.check(status, "ssp_exact_structure")
    return ex, st


def spgemm(A: DeviceCSR, A_val, B: DeviceCSR, B_val, row_cap, *, margin_pct: int = 0,
           spill_pct: int = 0, handle=None, stream=None, capacity=None):
    """Numeric C = A.B sized by per-row capacities (normally the prediction).

    ``ssp_spgemm_compute`` then ``ssp_spgemm_copy``: returns ``(C_rpt int64[M+1],
    C_col int32[nnz], C_val float64[nnz], info dict)``.  ``margin_pct`` enlarges
    every row's slot, ``spill_pct`` sizes the overflow area the rows share (a
    percentage of the slot entries).  ``capacity`` (entries of C to allocate)
    defaults to the exact NNZ(C) the compute call reports."""
    h = handle or default_handle(A.device)
    M = A.nrows
    dev = A.device
    for name, v, m in (("A_val", A_val, A), ("B_val", B_val, B)):
        if v.dtype != torch.float64 or v.numel() != m.nnz or v.device != dev:
            raise ValueError(f"{name} must be float64[{m.nnz}] on {dev}")
    if row_cap.dtype != torch.int64 or row_cap.numel() != M or row_cap.device != dev:
        raise ValueError(f"row_cap must be int64[{M}] on {dev}")
    C_rpt = torch.empty(M + 1, dtype=torch.int64, device=dev)
    info = _native.SspSpgemmInfo()
    a, b = A._c(), B._c()
    status = h._lib.ssp_spgemm_compute(h.ptr, ctypes.byref(a), A_val.data_ptr() if A.nnz else 0,
                                       ctypes.byref(b), B_val.data_ptr() if B.nnz else 0,
                                       row_cap.data_ptr() if M else 0, int(margin_pct),
                                       int(spill_pct), C_rpt.data_ptr(), ctypes.byref(info),
                                       _stream_ptr(stream))
    h.check(status, "ssp_spgemm_compute")
    nnz = int(info.nnz)
    cap = nnz if capacity is None else int(capacity)
    C_col = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    C_val = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
    status = h._lib.ssp_spgemm_copy(h.ptr, C_col.data_ptr(), C_val.data_ptr(), cap,
                                    _stream_ptr(stream))
    h.check(status, "ssp_spgemm_copy")
    return C_rpt, C_col[:nnz], C_val[:nnz], info.as_dict()


def kmv_estimate(A: DeviceCSR, B: DeviceCSR, sample_rate: float, k: int, seed: int, *,
                 handle=None, stream=None) -> dict:
    """The existing sampling estimator of related work (Amossen's k minimum
    values with BHash's row and column sampling): ``ssp_kmv_estimate``, a dict
    of its results."""
    h = handle or default_handle(A.device)
    out = _native.SspKmvResult()
    a, b = A._c(), B._c()
    status = h._lib.ssp_kmv_estimate(h.ptr, ctypes.byref(a), ctypes.byref(b), float(sample_rate),
                                     int(k), int(seed) % (1 << 64), ctypes.byref(out),
                                     _stream_ptr(stream))
    h.check(status, "ssp_kmv_estimate")
    return out.as_dict()


class Case:
    """One product of a batch and its device outputs (allocated here when not given)."""

    def __init__(self, A: DeviceCSR, B: DeviceCSR, sample_rate: float, seed: int, *,
                 sampler="bernoulli", return_row_flop: bool = False, out=None, stats=None):
        self.A, self.B = A, B
        self.sample_rate, self.seed, self.sampler = float(sample_rate), int(seed), sampler
        M = A.nrows
        self.pred = out if out is not None else torch.empty(M, dtype=torch.int64, device=A.device)
        self.row_flop = (torch.empty(M, dtype=torch.int64, device=A.device) if return_row_flop
                         else None)
        self.stats = stats if stats is not None else _new_stats(A.device)

    def _c(self) -> _native.SspCase:
        c = _native.SspCase()
        c.A, c.B = self.A._c(), self.B._c()
        c.sampler = _sampler_id(self.sampler)
        c.reserved = 0
        c.sample_rate = self.sample_rate
        c.seed = self.seed % (1 << 64)
        c.nnz_pred = self.pred.data_ptr() if self.A.nrows else 0
        c.row_flop = self.row_flop.data_ptr() if self.row_flop is not None and self.A.nrows else 0
        c.stats = self.stats.data_ptr() if self.stats is not None else 0
        return c


def _case_array(cases):
    arr = (_native.SspCase * max(len(cases), 1))()
    for i, c in enumerate(cases):
        arr[i] = c._c()
    return arr


def predict_batch(cases, *, handle=None, stream=None):
    """Predict every Case of `cases` with one launch sequence (ssp_predict_batch).

    Results land in each case's .pred / .row_flop / .stats; returns `cases`.
    """
    cases = list(cases)
    if not cases:
        return cases
    h = handle or default_handle(cases[0].A.device)
    arr = _case_array(cases)
    h.check(h._lib.ssp_predict_batch(h.ptr, len(cases), arr, _stream_ptr(stream)),
            "ssp_predict_batch")
    return cases


class BatchGraph:
    """A batch captured once as a HIP graph (ssp_batch_graph_*); launch() replays it."""

    def __init__(self, cases, *, handle=None):
        self.cases = list(cases)
        if not self.cases:
            raise ValueError("a batch graph needs at least one case")
        self.handle = handle or default_handle(self.cases[0].A.device)
        self._lib = self.handle._lib
        arr = _case_array(self.cases)
        g = ctypes.c_void_p()
        self.handle.check(self._lib.ssp_batch_graph_create(self.handle.ptr, len(self.cases), arr,
                                                           ctypes.byref(g)),
                          "ssp_batch_graph_create")
        self.ptr = g

    def launch(self, stream=None):
        self.handle.check(self._lib.ssp_batch_graph_launch(self.ptr, _stream_ptr(stream)),
                          "ssp_batch_graph_launch")
        return self.cases

    @property
    def workspace_bytes(self) -> int:
        return int(self._lib.ssp_batch_graph_workspace_bytes(self.ptr)) if self.ptr else 0

    def close(self):
        if self.ptr:
            self._lib.ssp_batch_graph_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_tuning() -> dict:
    """The library's default tuning (ssp_default_tuning) as a dict."""
    t = _native.SspTuning()
    _native.load().ssp_default_tuning(ctypes.byref(t))
    return t.as_dict()


def _tuning_struct(d: dict) -> "_native.SspTuning":
    t = _native.SspTuning()
    t.bin_max[:] = [int(x) for x in d["bin_max"]]
    t.hash_mult, t.long_len, t.big3 = int(d["hash_mult"]), int(d["long_len"]), int(d["big3"])
    t.split_target, t.est_max_rf = int(d["split_target"]), int(d["est_max_rf"])
    return t


def get_tuning(*, handle=None, device=None) -> dict:
    h = handle or default_handle(device)
    t = _native.SspTuning()
    h.check(h._lib.ssp_get_tuning(h.ptr, ctypes.byref(t)), "ssp_get_tuning")
    return t.as_dict()


def set_tuning(tuning: dict, *, handle=None, device=None):
    h = handle or default_handle(device)
    t = _tuning_struct(tuning)
    h.check(h._lib.ssp_set_tuning(h.ptr, ctypes.byref(t)), "ssp_set_tuning")


def autotune(cases, *, reps: int = 3, handle=None, stream=None) -> dict:
    """Tune the handle on a representative batch (ssp_autotune); returns
    {"tuning": ..., "best_ms": ..., "default_ms": ...}."""
    cases = list(cases)
    h = handle or default_handle(cases[0].A.device)
    arr = _case_array(cases)
    t = _native.SspTuning()
    best, dflt = ctypes.c_double(), ctypes.c_double()
    h.check(h._lib.ssp_autotune(h.ptr, len(cases), arr, int(reps), ctypes.byref(t),
                                ctypes.byref(best), ctypes.byref(dflt), _stream_ptr(stream)),
            "ssp_autotune")
    return {"tuning": t.as_dict(), "best_ms": best.value, "default_ms": dflt.value}


class Server:
    """Request server with continuous batching (ssp_server_*): register device
    matrices, submit predictions, poll or wait by ticket."""

    def __init__(self, *, handle=None, slots: int = 4, slot_bytes: int = 1 << 30,
                 max_batch: int = 64, device=None):
        self.handle = handle or default_handle(device)
        self._lib = self.handle._lib
        s = ctypes.c_void_p()
        self.handle.check(self._lib.ssp_server_create(self.handle.ptr, int(slots), int(slot_bytes),
                                                      int(max_batch), ctypes.byref(s)),
                          "ssp_server_create")
        self.ptr = s
        self._mats = []  # keep registered matrices alive

    def _check(self, status, where):
        if status != 0:
            raise SspError(status, where)

    def register(self, M: DeviceCSR) -> int:
        i = ctypes.c_int32()
        c = M._c()
        self._check(self._lib.ssp_server_register_matrix(self.ptr, ctypes.byref(c), ctypes.byref(i)),
                    "ssp_server_register_matrix")
        self._mats.append(M)
        return int(i.value)

    def submit(self, a: int, b: int, sample_rate: float, seed: int, out, stats=None,
               sampler="bernoulli") -> int:
        r = _native.SspRequest(int(a), int(b), _sampler_id(sampler), 0, float(sample_rate),
                               int(seed) % (1 << 64), out.data_ptr() if out.numel() else 0,
                               stats.data_ptr() if stats is not None else 0)
        t = ctypes.c_uint64()
        self._check(self._lib.ssp_server_submit(self.ptr, ctypes.byref(r), ctypes.byref(t)),
                    "ssp_server_submit")
        return int(t.value)

    def poll(self, ticket: int) -> bool:
        st = self._lib.ssp_server_poll(self.ptr, int(ticket))
        if st == -10:
            return False
        self._check(st, "ssp_server_poll")
        return True

    def wait(self, ticket: int, timeout: float = -1.0):
        self._check(self._lib.ssp_server_wait(self.ptr, int(ticket), float(timeout)),
                    "ssp_server_wait")

    def info(self) -> dict:
        o = _native.SspServerStats()
        self._check(self._lib.ssp_server_info(self.ptr, ctypes.byref(o)), "ssp_server_info")
        return {k: getattr(o, k) for k in _native.SERVER_STATS_FIELDS}

    def reset_stats(self):
        self._check(self._lib.ssp_server_reset_stats(self.ptr), "ssp_server_reset_stats")

    def close(self):
        if self.ptr:
            self._lib.ssp_server_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def validate_csr(M: DeviceCSR, *, handle=None, stream=None) -> int:
    """Number of CSR violations in M (synchronises)."""
    h = handle or default_handle(M.device)
    bad = torch.zeros(1, dtype=torch.int64, device=M.device)
    m = M._c()
    h.check(h._lib.ssp_validate_csr(h.ptr, ctypes.byref(m), bad.data_ptr(), _stream_ptr(stream)),
            "ssp_validate_csr")
    return int(bad.item())
