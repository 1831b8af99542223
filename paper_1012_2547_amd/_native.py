"""ctypes bindings to libsm.so (the C ABI in include/sm.h). Marshalling only."""
from __future__ import annotations

import ctypes
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsm.so")

SM_OK, SM_TRUNCATED, SM_EINVAL, SM_ENOMEM, SM_EDEVICE, SM_EBUSY = 0, 1, -1, -2, -3, -4
STATUS_NAMES = {0: "SM_OK", 1: "SM_TRUNCATED", -1: "SM_EINVAL", -2: "SM_ENOMEM",
                -3: "SM_EDEVICE", -4: "SM_EBUSY"}

ALGO_AUTO, ALGO_SHIFT_AND, ALGO_BNDM, ALGO_SBNDM, ALGO_HASHQ, ALGO_BLOCK, ALGO_BRUTE = 0, 1, 2, 3, 4, 5, 6
ALGO_FSBNDM = 7
ALGO_NAMES = {0: "auto", 1: "shift_and", 2: "bndm", 3: "sbndm", 4: "hashq", 5: "block", 6: "brute",
              7: "fsbndm"}


class SmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("lane_bytes", ctypes.c_int32), ("q", ctypes.c_int32),
                ("sigma_hint", ctypes.c_int32), ("tiles_per_wg", ctypes.c_int32),
                ("hbits", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("lane_bytes", ctypes.c_int32), ("q", ctypes.c_int32),
                ("hbits", ctypes.c_int32), ("tiles_per_wg", ctypes.c_int32),
                ("suffix", ctypes.c_int32)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("sigma_lo", ctypes.c_int32), ("sigma_hi", ctypes.c_int32),
                ("m_lo", ctypes.c_uint32), ("m_hi", ctypes.c_uint32), ("algo", ctypes.c_int32),
                ("lane_bytes", ctypes.c_int32), ("q", ctypes.c_int32),
                ("tiles_per_wg", ctypes.c_int32), ("hbits", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Prof(ctypes.Structure):
    _fields_ = [("calls", ctypes.c_uint64), ("count_ms", ctypes.c_double),
                ("emit_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("text_bytes", ctypes.c_uint64), ("sampled_calls", ctypes.c_uint64),
                ("sampled_count_ms", ctypes.c_double), ("batch_calls", ctypes.c_uint64),
                ("batch_ms", ctypes.c_double), ("filter_launches", ctypes.c_uint64),
                ("filter_ms", ctypes.c_double), ("filter_pattern_bytes", ctypes.c_uint64)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("pool_bytes", ctypes.c_uint64), ("host_bytes", ctypes.c_uint64),
                ("max_batch", ctypes.c_uint32), ("slots", ctypes.c_uint32),
                ("max_pending", ctypes.c_uint32), ("graphs_off", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 4)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("corpus", ctypes.c_uint32),
                ("count", ctypes.c_uint64), ("positions", ctypes.POINTER(ctypes.c_int64)),
                ("arrival_ns", ctypes.c_int64), ("start_ns", ctypes.c_int64),
                ("done_ns", ctypes.c_int64), ("batch_size", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class ServerMetrics(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("pending", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("batched_queries", ctypes.c_uint64),
                ("text_bytes", ctypes.c_uint64), ("out_bytes", ctypes.c_uint64),
                ("write_waves", ctypes.c_uint64), ("deferred", ctypes.c_uint64),
                ("p50_ns", ctypes.c_int64), ("p99_ns", ctypes.c_int64),
                ("p999_ns", ctypes.c_int64), ("max_ns", ctypes.c_int64),
                ("mean_ns", ctypes.c_double), ("span_ns", ctypes.c_int64),
                ("qps", ctypes.c_double), ("graph_launches", ctypes.c_uint64),
                ("graph_builds", ctypes.c_uint64), ("evicted", ctypes.c_uint64),
                ("evicted_bytes", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("mem_waits", ctypes.c_uint64), ("host_peak_bytes", ctypes.c_uint64),
                ("host_arena_bytes", ctypes.c_uint64)]


# every exported symbol and its prototype: (restype, argtypes)
_vp, _u64, _i32, _u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32
_pu64 = ctypes.POINTER(ctypes.c_uint64)
PROTOTYPES = {
    "sm_version": (ctypes.c_char_p, []),
    "sm_last_error": (ctypes.c_char_p, []),
    "sm_find_all": (_i32, [_vp, _u64, _vp, _u64, _vp, _u64, _pu64]),
    "sm_count": (_i32, [_vp, _u64, _vp, _u64, _pu64]),
    "sm_find_all_dev": (_i32, [_vp, _u64, _vp, _u64, _vp, _u64, _pu64, _vp]),
    "sm_count_dev": (_i32, [_vp, _u64, _vp, _u64, _pu64, _vp]),
    "sm_workspace_size": (_u64, [_u64, _u64, ctypes.POINTER(Opts)]),
    "sm_workspace_size_upto": (_u64, [_u64, _u64, ctypes.POINTER(Opts)]),
    "sm_find_all_async": (_i32, [_vp, _u64, _vp, _u64, _vp, _u64, _vp, _vp, _u64,
                                 ctypes.POINTER(Opts), _vp]),
    "sm_count_async": (_i32, [_vp, _u64, _vp, _u64, _vp, _vp, _u64, ctypes.POINTER(Opts), _vp]),
    "sm_find_all_noalloc": (_i32, [_vp, _u64, _vp, _u64, _vp, _u64, _vp, ctypes.POINTER(Opts), _vp]),
    "sm_plan_query": (_i32, [_vp, _u64, ctypes.POINTER(Opts), ctypes.POINTER(PlanInfo)]),
    "sm_corpus_open": (_i32, [_vp, _u64, _i32, ctypes.POINTER(_vp)]),
    "sm_corpus_close": (_i32, [_vp]),
    "sm_corpus_find_all": (_i32, [_vp, _vp, _u64, _vp, _u64, _pu64]),
    "sm_corpus_count": (_i32, [_vp, _vp, _u64, _pu64]),
    "sm_corpus_stats": (_i32, [_vp, _vp, ctypes.POINTER(ctypes.c_int32),
                                ctypes.POINTER(ctypes.c_double)]),
    "sm_corpus_find_all_async": (_i32, [_vp, _vp, _u64, _vp, _u64, _vp, _vp, _u64,
                                        ctypes.POINTER(Opts), _vp]),
    "sm_corpus_count_async": (_i32, [_vp, _vp, _u64, _vp, _vp, _u64, ctypes.POINTER(Opts), _vp]),
    "sm_tune_set": (_i32, [ctypes.POINTER(TuneEntry), _u32]),
    "sm_tune_get": (_i32, [ctypes.POINTER(TuneEntry), _u32, ctypes.POINTER(ctypes.c_uint32)]),
    "sm_corpus_text": (_i32, [_vp, ctypes.POINTER(_vp), _pu64]),
    "sm_batch_workspace_size": (_u64, [_vp, _vp, _vp, _u32]),
    "sm_batch_count": (_i32, [_vp, _vp, _vp, _u32, _vp]),
    "sm_batch_find_all": (_i32, [_vp, _vp, _vp, _u32, _vp, _u64, _vp]),
    "sm_batch_count_async": (_i32, [_vp, _vp, _vp, _u32, _vp, _vp, _u64, _vp]),
    "sm_batch_find_all_async": (_i32, [_vp, _vp, _vp, _u32, _vp, _u64, _vp, _vp, _u64, _vp]),
    "sm_batch_open": (_i32, [_vp, _vp, _vp, _u32, ctypes.POINTER(_vp)]),
    "sm_batch_offsets": (_i32, [_vp, _vp]),
    "sm_batch_write_async": (_i32, [_vp, _u64, _u64, _vp, _vp]),
    "sm_batch_close": (_i32, [_vp]),
    "sm_batch_set_wave_bytes": (_i32, [_u64]),
    "sm_batch_set_write_policy": (_i32, [_i32]),
    "sm_now_ns": (ctypes.c_int64, []),
    "sm_server_create": (_i32, [ctypes.POINTER(ServerConfig), ctypes.POINTER(_vp)]),
    "sm_server_add_corpus": (_i32, [_vp, _vp, ctypes.POINTER(ctypes.c_uint32)]),
    "sm_server_submit": (_i32, [_vp, _u32, _vp, _u64, ctypes.c_int64, _pu64]),
    "sm_server_wait": (_i32, [_vp, _u64, ctypes.c_int64, ctypes.POINTER(Result)]),
    "sm_server_poll": (_i32, [_vp, _u64, ctypes.POINTER(Result)]),
    "sm_result_free": (_i32, [_vp, _u64]),
    "sm_server_stats": (_i32, [_vp, ctypes.POINTER(ServerMetrics)]),
    "sm_server_reset_stats": (_i32, [_vp]),
    "sm_server_destroy": (_i32, [_vp]),
    "sm_prof_enable": (_i32, [_i32]),
    "sm_prof_collect": (_i32, [ctypes.POINTER(Prof)]),
}

_lock = threading.Lock()
_lib = None


def load(path: str = LIB_PATH):
    """Load libsm.so. Raises ImportError when the library has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise ImportError("libsm.so is not built (%s); run "
                                  "`python -m paper_1012_2547_amd.build`" % path)
            L = ctypes.CDLL(path)
            for name, (res, args) in PROTOTYPES.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
    return _lib


def last_error() -> str:
    return load().sm_last_error().decode(errors="replace")


def check(status: int, allow_truncated: bool = True) -> int:
    if status < 0 or (status == SM_TRUNCATED and not allow_truncated):
        raise SmError(status, last_error())
    return status
