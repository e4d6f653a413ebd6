"""ctypes view of the C ABI in include/tds.h (argument marshalling only).

Loading fails loudly when libtds.so has not been built: there is no CPU
fallback anywhere in this package.
"""
from __future__ import annotations

import ctypes as C
import os
from pathlib import Path

PKG = Path(__file__).resolve().parent
LIB_PATH = Path(os.environ.get("TDS_LIB", PKG / "libtds.so"))

TDS_OK = 0
TDS_EINVAL = -1
TDS_ENOMEM = -2
TDS_EDEVICE = -3
TDS_EOVERFLOW = -4
TDS_ESTATE = -5
TDS_EBUSY = -6

TDS_MEM_HOST = 0
TDS_MEM_DEVICE = 1
TDS_MODE_FP64 = 0
TDS_MODE_FP32_REFINE = 1
TDS_TILE_PERIODIC = 0
TDS_TILE_RANGE = 1
TDS_TILE_GREEDY_MIN = 2
TDS_TILE_GREEDY_MAX = 3
TDS_QF_TIMING = 1
TDS_QF_COUNT_OVERLAP = 2
TDS_QF_KERNEL_OVERLAP = 4
TDS_QF_TIMING_PAIR = 8
TDS_NOALLOC_SCRATCH_BYTES = 64 << 20

_P = C.c_void_p


class tds_segments(C.Structure):
    _fields_ = [("n", C.c_int64), ("mem", C.c_int32), ("reserved", C.c_int32),
                ("x0", _P), ("y0", _P), ("z0", _P), ("t0", _P),
                ("x1", _P), ("y1", _P), ("z1", _P), ("t1", _P),
                ("traj_id", _P)]


class tds_index_opts(C.Structure):
    _fields_ = [("num_bins", C.c_int32), ("flags", C.c_int32)]


class tds_query_opts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("tiling", C.c_int32), ("batch_size", C.c_int32),
                ("block_size", C.c_int32), ("reserved0", C.c_int32), ("max_retries", C.c_int32),
                ("capacity", C.c_int64), ("grid", C.c_int32), ("flags", C.c_int32)]


class tds_hit(C.Structure):
    _fields_ = [("query_idx", C.c_int64), ("entry_idx", C.c_int64), ("entry_traj", C.c_int64),
                ("t_a", C.c_double), ("t_b", C.c_double)]


class tds_traj_hit(C.Structure):
    _fields_ = [("query_traj", C.c_int64), ("entry_traj", C.c_int64), ("t_a", C.c_double),
                ("t_b", C.c_double)]


class tds_tile_info(C.Structure):
    _fields_ = [("q_first", C.c_int32), ("n_query", C.c_int32), ("e_first", C.c_int32),
                ("n_entry", C.c_int32)]


class tds_stats(C.Structure):
    _fields_ = [("n_query", C.c_int64), ("n_eval", C.c_int64), ("n_overlap", C.c_int64),
                ("n_overlap_k", C.c_int64), ("n_refine", C.c_int64), ("n_hit", C.c_int64),
                ("n_tiles", C.c_int64), ("n_items", C.c_int64), ("retries", C.c_int32),
                ("grid", C.c_int32), ("ms_prep", C.c_float), ("ms_pair", C.c_float),
                ("ms_fetch", C.c_float), ("ms_refine", C.c_float), ("chunk", C.c_int32),
                ("reserved1", C.c_int32)]


class tds_index_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("num_bins", C.c_int32), ("nonempty_bins", C.c_int32),
                ("t_first", C.c_double), ("t_last", C.c_double), ("bin_width", C.c_double),
                ("device_bytes", C.c_int64)]


class tds_bin(C.Structure):
    _fields_ = [("start", C.c_double), ("end", C.c_double), ("first", C.c_int64),
                ("last", C.c_int64), ("bin", C.c_int64)]


class tds_server_opts(C.Structure):
    _fields_ = [("streams", C.c_int32), ("max_batch_segments", C.c_int32), ("max_waiting", C.c_int64),
                ("pool_bytes", C.c_double), ("k_safety", C.c_double), ("epochs", C.c_int32),
                ("reserve_segments", C.c_int32), ("alpha_prior", C.c_double), ("query", tds_query_opts)]


class tds_request_info(C.Structure):
    _fields_ = [("arrival", C.c_double), ("admit", C.c_double), ("done", C.c_double),
                ("n_hit", C.c_int64), ("batch", C.c_int64), ("status", C.c_int32),
                ("n_batch_requests", C.c_int32)]


class tds_server_stats(C.Structure):
    _fields_ = [("batches", C.c_int64), ("requests_done", C.c_int64), ("retries", C.c_int64),
                ("segments", C.c_int64), ("device_bytes", C.c_int64), ("busy_s", C.c_double),
                ("stage_s", C.c_double), ("wait_s", C.c_double), ("split_s", C.c_double)]


# name -> (restype, argtypes); every symbol include/tds.h declares
# tds_alloc_fn / tds_free_fn
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)

SIGNATURES = {
    "tds_build_index": (C.c_int, [C.POINTER(tds_segments), C.POINTER(tds_index_opts), _P, C.POINTER(_P)]),
    "tds_index_info_get": (C.c_int, [_P, C.POINTER(tds_index_info)]),
    "tds_index_bins": (C.c_int, [_P, C.POINTER(tds_bin), C.c_int64, C.POINTER(C.c_int64)]),
    "tds_index_destroy": (None, [_P]),
    "tds_plan_bins": (C.c_int, [_P, _P, C.c_int64, C.c_int32, C.POINTER(tds_bin), C.c_int64,
                                C.POINTER(C.c_int64)]),
    "tds_plan_ranges": (C.c_int, [C.POINTER(tds_bin), C.c_int64, _P, _P, C.c_int64, _P, _P]),
    "tds_query_create": (C.c_int, [_P, C.POINTER(_P)]),
    "tds_query_destroy": (None, [_P]),
    "tds_query_batch": (C.c_int, [_P, C.POINTER(tds_segments), _P, C.POINTER(tds_query_opts), _P]),
    "tds_fetch_results": (C.c_int, [_P, _P, C.c_int64, C.c_int32, C.POINTER(C.c_int64)]),
    "tds_query_stats": (C.c_int, [_P, C.POINTER(tds_stats)]),
    "tds_fetch_trajectories": (C.c_int, [_P, _P, C.c_int32, _P, C.c_int64, C.c_int32,
                                         C.POINTER(C.c_int64)]),
    "tds_query_ranges": (C.c_int, [_P, _P, _P, C.c_int64]),
    "tds_index_times": (C.c_int, [_P, _P, _P, C.c_int64]),
    "tds_query_tiles": (C.c_int, [_P, _P, C.c_int64, _P, C.c_int64, C.POINTER(C.c_int64),
                                  C.POINTER(C.c_int64)]),
    "tds_set_allocator": (C.c_int, [ALLOC_FN, FREE_FN, _P]),
    "tds_search_noalloc": (C.c_int, [_P, C.POINTER(tds_segments), _P, C.POINTER(tds_query_opts), _P,
                                     C.c_int64, C.POINTER(C.c_int64), _P]),
    "tds_query_reserve": (C.c_int, [_P, C.c_int64, C.c_int64, C.POINTER(tds_query_opts)]),
    "tds_query_device_bytes": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "tds_server_create": (C.c_int, [_P, C.POINTER(tds_server_opts), C.POINTER(_P)]),
    "tds_server_now": (C.c_double, [_P]),
    "tds_server_submit": (C.c_int, [_P, C.POINTER(tds_segments), _P, C.c_double, C.POINTER(C.c_int64)]),
    "tds_server_wait": (C.c_int, [_P, C.c_int64, C.c_double, C.POINTER(tds_request_info)]),
    "tds_server_results": (C.c_int, [_P, C.c_int64, _P, C.c_int64, C.POINTER(C.c_int64)]),
    "tds_server_release": (C.c_int, [_P, C.c_int64]),
    "tds_server_stats_get": (C.c_int, [_P, C.POINTER(tds_server_stats)]),
    "tds_server_alpha": (C.c_int, [_P, _P, C.c_int32, C.POINTER(C.c_int32)]),
    "tds_server_destroy": (None, [_P]),
    "tds_last_error": (C.c_char_p, []),
    "tds_abi_version": (C.c_int, []),
}

_lib = None


class TdsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tds error {code}: {msg}")
        self.code = code


def lib():
    """The loaded library; raises if libtds.so is missing (no fallback)."""
    global _lib
    if _lib is None:
        # torch carries its own HIP runtime; load it before libtds.so so that
        # the process holds exactly one HIP runtime (libtds then binds to it).
        import torch  # noqa: F401
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(str(LIB_PATH))
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != TDS_OK:
        raise TdsError(rc, lib().tds_last_error().decode(errors="replace"))
    return rc
