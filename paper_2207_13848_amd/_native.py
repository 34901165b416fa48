"""ctypes declarations of the C ABI in include/ssp.h (libssp.so, built in-tree).

No fallback: if the HIP library is missing, loading fails with an error that
names the build step.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libssp.so")

SSP_OK = 0
STATUS_NAMES = {
    0: "SSP_OK", -1: "SSP_ERR_INVALID_ARG", -2: "SSP_ERR_DIM_MISMATCH", -3: "SSP_ERR_OVERFLOW",
    -4: "SSP_ERR_BUDGET", -5: "SSP_ERR_OOM", -6: "SSP_ERR_HIP", -7: "SSP_ERR_NO_DEVICE",
    -8: "SSP_ERR_INVALID_CSR", -9: "SSP_ERR_BUSY", -10: "SSP_ERR_NOT_READY",
}
SAMPLER_BERNOULLI, SAMPLER_PAPER = 0, 1
FLAG_EMPTY_SAMPLE, FLAG_SATURATED = 1, 2

# every symbol include/ssp.h declares (checked by the ABI tests)
EXPORTED = (
    "ssp_create", "ssp_destroy", "ssp_workspace_bytes", "ssp_predict_structure",
    "ssp_predict_structure_ex", "ssp_reference_estimate", "ssp_exact_structure",
    "ssp_validate_csr", "ssp_status_string", "ssp_last_error", "ssp_version",
    "ssp_timing_enable", "ssp_timing_read", "ssp_predict_batch", "ssp_batch_graph_create",
    "ssp_batch_graph_launch", "ssp_batch_graph_workspace_bytes", "ssp_batch_graph_destroy",
    "ssp_server_create", "ssp_server_register_matrix", "ssp_server_submit", "ssp_server_poll",
    "ssp_server_wait", "ssp_server_info", "ssp_server_reset_stats", "ssp_server_destroy",
    "ssp_default_tuning", "ssp_get_tuning", "ssp_set_tuning", "ssp_autotune",
    "ssp_spgemm_compute", "ssp_spgemm_copy", "ssp_kmv_estimate",
    "ssp_predict_structure_noalloc",
)


class SspCsr(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rpt", ctypes.c_void_p), ("col", ctypes.c_void_p)]


class SspCase(ctypes.Structure):
    _fields_ = [("A", SspCsr), ("B", SspCsr), ("sampler", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("sample_rate", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("nnz_pred", ctypes.c_void_p),
                ("row_flop", ctypes.c_void_p), ("stats", ctypes.c_void_p)]


class SspSpgemmInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("nnz", "total_flop", "slot_entries", "overflow_rows", "overflow_nnz",
                 "slot_bytes", "spill_rows", "spill_nnz", "spill_bytes")]

    def as_dict(self) -> dict:
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class SspKmvResult(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in
                ("rows_kept", "cols_kept", "products", "distinct_kept", "kth_hash", "k",
                 "threshold")] + [("nnz_sample", ctypes.c_double), ("nnz_estimate", ctypes.c_double)]

    def as_dict(self) -> dict:
        d = {n: getattr(self, n) for n, _ in self._fields_}
        d = {n: (int(v) if isinstance(v, int) else float(v)) for n, v in d.items()}
        if d["nnz_estimate"] < 0:
            d["nnz_estimate"] = None
        return d


class SspTuning(ctypes.Structure):
    _fields_ = [("bin_max", ctypes.c_uint32 * 3), ("hash_mult", ctypes.c_uint32),
                ("long_len", ctypes.c_uint32), ("big3", ctypes.c_int32),
                ("split_target", ctypes.c_uint64), ("est_max_rf", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {"bin_max": list(self.bin_max), "hash_mult": self.hash_mult,
                "long_len": self.long_len, "big3": self.big3, "split_target": self.split_target,
                "est_max_rf": self.est_max_rf}


class SspRequest(ctypes.Structure):
    _fields_ = [("a", ctypes.c_int32), ("b", ctypes.c_int32), ("sampler", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("sample_rate", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("nnz_pred", ctypes.c_void_p),
                ("stats", ctypes.c_void_p)]


SERVER_STATS_FIELDS = ("submitted", "completed", "batches", "max_batch_seen", "queued",
                       "max_slots_busy", "elapsed_s", "latency_p50_ms", "latency_p99_ms",
                       "latency_mean_ms", "latency_max_ms")


class SspServerStats(ctypes.Structure):
    _fields_ = ([(n, ctypes.c_uint64) for n in SERVER_STATS_FIELDS[:6]] +
                [(n, ctypes.c_double) for n in SERVER_STATS_FIELDS[6:]])


STATS_FIELDS = ("total_flop", "n_sampled", "sample_flop", "sample_nnz", "out_sum", "nrows",
                "flags", "a_sample_nnz")


class SspStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in STATS_FIELDS]


class SspPhaseTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_uint64),
                ("total_ms", ctypes.c_double)]


class SspError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        msg = f"{where}: {STATUS_NAMES.get(status, status)}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)


_lib = None


def load():
    """Load libssp.so, declaring argument types.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, u64, dbl, cint = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double,
                               ctypes.c_int)
    csr_p = ctypes.POINTER(SspCsr)
    lib.ssp_create.argtypes = [ctypes.POINTER(vp), cint, ctypes.c_size_t]
    lib.ssp_destroy.argtypes = [vp]
    lib.ssp_workspace_bytes.argtypes = [vp]
    lib.ssp_workspace_bytes.restype = ctypes.c_size_t
    lib.ssp_predict_structure.argtypes = [vp, csr_p, csr_p, dbl, u64, vp, vp, vp, vp]
    lib.ssp_predict_structure_ex.argtypes = [vp, csr_p, csr_p, cint, dbl, u64, vp, vp, vp, vp]
    lib.ssp_predict_structure_noalloc.argtypes = [vp, csr_p, csr_p, cint, dbl, u64, vp, vp, vp,
                                                  vp]
    lib.ssp_reference_estimate.argtypes = [vp, csr_p, csr_p, cint, dbl, u64, vp, vp, vp]
    lib.ssp_exact_structure.argtypes = [vp, csr_p, csr_p, vp, vp, vp]
    lib.ssp_validate_csr.argtypes = [vp, csr_p, vp, vp]
    for f in ("ssp_create", "ssp_destroy", "ssp_predict_structure", "ssp_predict_structure_ex",
              "ssp_predict_structure_noalloc",
              "ssp_reference_estimate", "ssp_exact_structure", "ssp_validate_csr"):
        getattr(lib, f).restype = cint
    lib.ssp_status_string.argtypes = [cint]
    lib.ssp_status_string.restype = ctypes.c_char_p
    lib.ssp_last_error.argtypes = [vp]
    lib.ssp_last_error.restype = ctypes.c_char_p
    lib.ssp_timing_enable.argtypes = [vp, cint]
    lib.ssp_timing_enable.restype = cint
    lib.ssp_timing_read.argtypes = [vp, ctypes.POINTER(SspPhaseTime), cint]
    lib.ssp_timing_read.restype = cint
    case_p = ctypes.POINTER(SspCase)
    lib.ssp_predict_batch.argtypes = [vp, cint, case_p, vp]
    lib.ssp_batch_graph_create.argtypes = [vp, cint, case_p, ctypes.POINTER(vp)]
    lib.ssp_batch_graph_launch.argtypes = [vp, vp]
    lib.ssp_batch_graph_workspace_bytes.argtypes = [vp]
    lib.ssp_batch_graph_workspace_bytes.restype = ctypes.c_size_t
    lib.ssp_batch_graph_destroy.argtypes = [vp]
    u64 = ctypes.c_uint64
    lib.ssp_server_create.argtypes = [vp, cint, ctypes.c_size_t, cint, ctypes.POINTER(vp)]
    lib.ssp_server_register_matrix.argtypes = [vp, csr_p, ctypes.POINTER(ctypes.c_int32)]
    lib.ssp_server_submit.argtypes = [vp, ctypes.POINTER(SspRequest), ctypes.POINTER(u64)]
    lib.ssp_server_poll.argtypes = [vp, u64]
    lib.ssp_server_wait.argtypes = [vp, u64, dbl]
    lib.ssp_server_info.argtypes = [vp, ctypes.POINTER(SspServerStats)]
    lib.ssp_server_reset_stats.argtypes = [vp]
    lib.ssp_server_destroy.argtypes = [vp]
    tun_p = ctypes.POINTER(SspTuning)
    lib.ssp_default_tuning.argtypes = [tun_p]
    lib.ssp_default_tuning.restype = None
    lib.ssp_get_tuning.argtypes = [vp, tun_p]
    lib.ssp_set_tuning.argtypes = [vp, tun_p]
    lib.ssp_autotune.argtypes = [vp, cint, case_p, cint, tun_p, ctypes.POINTER(dbl),
                                 ctypes.POINTER(dbl), vp]
    lib.ssp_version.argtypes = []
    lib.ssp_version.restype = ctypes.c_char_p
    lib.ssp_spgemm_compute.argtypes = [vp, csr_p, vp, csr_p, vp, vp, ctypes.c_int32, ctypes.c_int32,
                                       vp, ctypes.POINTER(SspSpgemmInfo), vp]
    lib.ssp_spgemm_compute.restype = cint
    lib.ssp_spgemm_copy.argtypes = [vp, vp, vp, ctypes.c_int64, vp]
    lib.ssp_spgemm_copy.restype = cint
    lib.ssp_kmv_estimate.argtypes = [vp, csr_p, csr_p, dbl, ctypes.c_uint32, u64,
                                     ctypes.POINTER(SspKmvResult), vp]
    lib.ssp_kmv_estimate.restype = cint
    _lib = lib
    return lib
