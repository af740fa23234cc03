"""ctypes declarations of libdlmi.so (the C ABI in include/dlmi.h).

Argument marshalling only.  Loading fails loudly when the library has not
been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdlmi.so")

DL_OK, DL_ERR_INVALID, DL_ERR_OOM, DL_ERR_CAPACITY, DL_ERR_WORKSPACE, DL_ERR_DEVICE, DL_ERR_BUSY, DL_ERR_CANCELLED = range(8)
STATUS_NAMES = {0: "DL_OK", 1: "DL_ERR_INVALID", 2: "DL_ERR_OOM", 3: "DL_ERR_CAPACITY", 4: "DL_ERR_WORKSPACE",
                5: "DL_ERR_DEVICE", 6: "DL_ERR_BUSY", 7: "DL_ERR_CANCELLED"}
PREC = {"fp32": 0, "bf16": 1, "fp16": 2, "fp8": 3}
NUM_STAGES = 7
STAGES = ["featurize", "prep", "contract", "recheck", "sort", "select", "index"]


class dl_mat(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("n", ctypes.c_int64), ("d", ctypes.c_int32), ("ld", ctypes.c_int64)]


class dl_pairs(ctypes.Structure):
    _fields_ = [("i", ctypes.c_void_p), ("j", ctypes.c_void_p), ("dist", ctypes.c_void_p),
                ("capacity", ctypes.c_int64), ("count", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("ties", ctypes.c_int64)]


class dl_box(ctypes.Structure):
    _fields_ = [("frame", ctypes.c_int32), ("x0", ctypes.c_int32), ("y0", ctypes.c_int32), ("x1", ctypes.c_int32),
                ("y1", ctypes.c_int32)]


class dl_index_info(ctypes.Structure):
    _fields_ = [("tiles_total", ctypes.c_int64), ("tiles_computed", ctypes.c_int64), ("pivots", ctypes.c_int32),
                ("ksteps_per_tile", ctypes.c_int32), ("ksteps_computed", ctypes.c_int64)]


class dl_peaks(ctypes.Structure):
    _fields_ = [("mfma_fp32_tflops", ctypes.c_double), ("mfma_bf16_tflops", ctypes.c_double),
                ("mfma_fp16_tflops", ctypes.c_double), ("mfma_fp8_tflops", ctypes.c_double),
                ("hbm_copy_gbps", ctypes.c_double), ("mfma_bf16_2w_tflops", ctypes.c_double),
                ("mfma_bf16_32x32_2w_tflops", ctypes.c_double), ("hbm_read_gbps", ctypes.c_double),
                ("mfma_bf16_lds_tflops", ctypes.c_double)]


class dl_topk_info(ctypes.Structure):
    _fields_ = [("band_entries", ctypes.c_int64), ("ties", ctypes.c_int64)]


class dl_server_config(ctypes.Structure):
    _fields_ = [("n_streams", ctypes.c_int32), ("max_batch_requests", ctypes.c_int32),
                ("max_batch_rows", ctypes.c_int64), ("pairs_per_row", ctypes.c_int64), ("band_cap", ctypes.c_int32),
                ("small_rows", ctypes.c_int64)]


class dl_request(ctypes.Structure):
    _fields_ = [("query", dl_mat), ("mode", ctypes.c_int32), ("eps", ctypes.c_double), ("k", ctypes.c_int32)]


class dl_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("mode", ctypes.c_int32), ("rows", ctypes.c_int64), ("k", ctypes.c_int32),
                ("i", ctypes.c_void_p), ("j", ctypes.c_void_p), ("dist", ctypes.c_void_p), ("count", ctypes.c_int64),
                ("queued_ms", ctypes.c_double), ("latency_ms", ctypes.c_double), ("batch_id", ctypes.c_int64),
                ("batch_requests", ctypes.c_int32)]


class dl_server_info(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("cancelled", ctypes.c_int64), ("batches", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("mean_batch_requests", ctypes.c_double), ("pairs_done", ctypes.c_double),
                ("span_ms", ctypes.c_double), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("arena_in_use", ctypes.c_size_t), ("arena_peak", ctypes.c_size_t),
                ("batch_ms", ctypes.c_double), ("batch_pairs", ctypes.c_double)]


DL_MODE_EPS, DL_MODE_TOPK = 0, 1
NOALLOC_SCRATCH_BYTES = 64 << 20  # DL_NOALLOC_SCRATCH_BYTES

# name -> (restype, argtypes); every symbol include/dlmi.h declares
P, i32, i64, f64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
SIGNATURES = {
    "dl_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(P)]),
    "dl_destroy": (None, [P]),
    "dl_last_error": (ctypes.c_char_p, [P]),
    "dl_version": (ctypes.c_char_p, []),
    "dl_set_timing": (ctypes.c_int, [P, ctypes.c_int]),
    "dl_get_timing": (ctypes.c_int, [P, P, P, ctypes.c_int]),
    "dl_featurize_rgb8": (ctypes.c_int, [P, P, i64, i32, i32, i32, P, P]),
    "dl_featurize_crops_rgb8": (ctypes.c_int, [P, P, i64, i32, i32, P, i64, i32, P, P]),
    "dl_pair_d2": (ctypes.c_int, [P, dl_mat, dl_mat, P, P, i64, P, P]),
    "dl_join_eps_workspace": (sz, [i64, i64, i32, ctypes.c_int, ctypes.c_int, i64]),
    "dl_join_eps": (ctypes.c_int, [P, dl_mat, dl_mat, ctypes.c_int, f64, ctypes.c_int, P, sz,
                                   ctypes.POINTER(dl_pairs), P]),
    "dl_required_workspace": (sz, [P]),
    "dl_join_eps_noalloc": (ctypes.c_int, [P, dl_mat, dl_mat, ctypes.c_int, f64, ctypes.c_int,
                                           ctypes.POINTER(dl_pairs), P]),
    "dl_join_eps_indexed_workspace": (sz, [i64, i64, i32, ctypes.c_int, ctypes.c_int, i64, i32]),
    "dl_join_eps_indexed": (ctypes.c_int, [P, dl_mat, dl_mat, ctypes.c_int, f64, ctypes.c_int, i32, P, sz,
                                           ctypes.POINTER(dl_pairs), ctypes.POINTER(dl_index_info), P]),
    "dl_join_eps_filtered_workspace": (sz, [i64, i64, i32, ctypes.c_int, ctypes.c_int, i32, i64, i64]),
    "dl_join_eps_filtered": (ctypes.c_int, [P, dl_mat, dl_mat, ctypes.c_int, f64, ctypes.c_int, P, P, i32, i32, i64,
                                            i64, P, sz, ctypes.POINTER(dl_pairs), P]),
    "dl_join_topk_workspace": (sz, [i64, i64, i32, ctypes.c_int, ctypes.c_int, i32, i32]),
    "dl_join_topk": (ctypes.c_int, [P, dl_mat, dl_mat, ctypes.c_int, i32, ctypes.c_int, ctypes.c_int, i32, P, sz,
                                    P, P, ctypes.POINTER(dl_topk_info), P]),
    "dl_join_topk_indexed_workspace": (sz, [i64, i64, i32, ctypes.c_int, ctypes.c_int, ctypes.c_int, i32, i32, i32]),
    "dl_join_topk_indexed": (ctypes.c_int, [P, dl_mat, dl_mat, ctypes.c_int, i32, ctypes.c_int, ctypes.c_int, i32,
                                            i32, P, sz, P, P, ctypes.POINTER(dl_topk_info),
                                            ctypes.POINTER(dl_index_info), P]),
    "dl_store_bytes": (sz, [i64, i32, ctypes.c_int]),
    "dl_store_create": (ctypes.c_int, [P, dl_mat, ctypes.c_int, P, sz, ctypes.POINTER(P), P]),
    "dl_store_destroy": (None, [P]),
    "dl_store_rows": (i64, [P]),
    "dl_join_eps_store_workspace": (sz, [i64, P, i64]),
    "dl_join_eps_store": (ctypes.c_int, [P, dl_mat, P, f64, P, sz, ctypes.POINTER(dl_pairs), P]),
    "dl_store_featurize_rgb8": (ctypes.c_int, [P, P, i64, i32, i32, P, i64, i32, ctypes.c_int, P, P, sz,
                                               ctypes.POINTER(P), P]),
    "dl_join_eps_store_self_workspace": (sz, [P, i64]),
    "dl_join_eps_store_self": (ctypes.c_int, [P, P, f64, P, sz, ctypes.POINTER(dl_pairs), P]),
    "dl_join_topk_store_workspace": (sz, [i64, P, i32, i32]),
    "dl_join_topk_store": (ctypes.c_int, [P, dl_mat, P, i32, i32, P, sz, P, P, ctypes.POINTER(dl_topk_info), P]),
    "dl_server_create": (ctypes.c_int, [ctypes.c_int, P, ctypes.POINTER(dl_server_config), P, sz, ctypes.POINTER(P)]),
    "dl_server_submit": (ctypes.c_int, [P, ctypes.POINTER(dl_request), ctypes.POINTER(ctypes.c_uint64)]),
    "dl_server_wait": (ctypes.c_int, [P, ctypes.c_uint64, i32, ctypes.POINTER(dl_result)]),
    "dl_server_release": (ctypes.c_int, [P, ctypes.c_uint64]),
    "dl_server_cancel": (ctypes.c_int, [P, ctypes.c_uint64]),
    "dl_server_stats": (ctypes.c_int, [P, ctypes.POINTER(dl_server_info)]),
    "dl_server_reset_stats": (ctypes.c_int, [P]),
    "dl_server_destroy": (None, [P]),
    "dl_measure_peaks": (ctypes.c_int, [P, ctypes.POINTER(dl_peaks)]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libdlmi.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libdlmi.so is not built (run `python -c 'import __graft_entry__ as g; g.build()'` "
                               "or `python paper_1812_07607_amd/build.py`); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class DLError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status
