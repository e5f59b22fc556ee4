"""ctypes declarations of the C ABI in include/ann.h (argument marshalling only).

The shared library must have been built (``python -m paper_1312_3062_amd.build``);
importing the package without it raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libann.so")

ANN_U8, ANN_F32 = 0, 1
ANN_OK, ANN_EINVAL, ANN_ENOMEM, ANN_EDEVICE, ANN_ESTATE, ANN_EUNSUPPORTED, ANN_EIO, ANN_ERESOURCE = (
    0, -1, -2, -3, -4, -5, -6, -7)
PRECISION_EXACT, PRECISION_BF16_RERANK = 0, 1
NSTATS = 12
STAT_NAMES = ("evals", "ref_pops", "bridge_pops", "bridge_ids", "bridges_gen", "heap_max", "flags", "rows",
              "lookaheads", "rerun", "moved", "reserved11")


class BuildParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("graph_k", C.c_int32), ("P", C.c_int32), ("K", C.c_int32),
                ("kmeans_iters", C.c_int32), ("bridge_t", C.c_int32), ("bridge_b", C.c_int32),
                ("reserved", C.c_int32), ("seed", C.c_uint64)]


class SearchParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("queue_len", C.c_int32), ("precision", C.c_int32),
                ("rerank_k", C.c_int32), ("lookahead", C.c_int32), ("persistent", C.c_int32),
                ("waves_per_cu", C.c_int32), ("order", C.c_int32)]


class IndexInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int32), ("dtype", C.c_int32), ("P", C.c_int32), ("K", C.c_int32),
                ("graph_k", C.c_int32), ("reserved", C.c_int32), ("n_bridges", C.c_int64),
                ("n_bridge_entries", C.c_int64), ("device_bytes", C.c_int64)]


class ServerParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("slots", C.c_int32), ("slot_queries", C.c_int32), ("kmax", C.c_int32),
                ("max_budget", C.c_int32), ("lds_rounds", C.c_int32), ("device_bytes", C.c_int64),
                ("search", SearchParams)]


class ServerInfo(C.Structure):
    _fields_ = [("pending", C.c_int64), ("busy_slots", C.c_int64), ("launches", C.c_int64),
                ("lds_in_flight", C.c_int64), ("lds_limit", C.c_int64), ("device_in_flight", C.c_int64),
                ("device_bytes", C.c_int64)]


class IvfParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("lists", C.c_int32), ("pq_m", C.c_int32), ("pq_iters", C.c_int32),
                ("assign_budget", C.c_int32), ("reserved", C.c_int32), ("seed", C.c_uint64),
                ("centres", BuildParams)]


class IvfInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int32), ("lists", C.c_int32), ("pq_m", C.c_int32),
                ("reserved", C.c_int32), ("device_bytes", C.c_int64)]


class AnnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


_lib = None

# every exported symbol of include/ann.h and its (restype, argtypes)
_vp, _i64, _i32, _cp = C.c_void_p, C.c_int64, C.c_int32, C.c_char_p
SIGNATURES = {
    "ann_build_index": (_i32, [_vp, _i64, _i32, _i32, C.POINTER(BuildParams), _vp, _vp, C.POINTER(_vp)]),
    "ann_index_import": (_i32, [_vp, _i64, _i32, _i32, _i32, _i32, _vp, _i32, _vp, _vp, _vp, C.POINTER(_vp)]),
    "ann_index_get_info": (_i32, [_vp, C.POINTER(IndexInfo)]),
    "ann_index_export": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "ann_index_save": (_i32, [_vp, _cp]),
    "ann_index_load": (_i32, [_cp, C.POINTER(_vp)]),
    "ann_index_free": (None, [_vp]),
    "ann_search": (_i32, [_vp, _vp, _i64, _i32, _i32, C.POINTER(SearchParams), _vp, _vp]),
    "ann_search_device": (_i32, [_vp, _vp, _i64, _i32, _i32, _vp, _vp, C.POINTER(SearchParams), _vp, _vp, _vp,
                                 _vp, _vp]),
    "ann_search_workspace_size": (_i32, [_vp, _i64, _i32, _i32, C.POINTER(SearchParams), C.POINTER(_i64)]),
    "ann_search_device_ws": (_i32, [_vp, _vp, _i64, _i32, _i32, _vp, _vp, C.POINTER(SearchParams), _vp, _vp, _vp,
                                    _vp, _vp, _i64, _vp]),
    "ann_search_graph_device": (_i32, [_vp, _vp, _i64, _i32, _i32, _vp, _i32, C.POINTER(SearchParams), _vp, _vp,
                                       _vp, _vp, _vp]),
    "ann_search_device_noalloc": (_i32, [_vp, _vp, _i64, _i32, _i32, _vp, _vp, C.POINTER(SearchParams), _vp, _vp,
                                         _vp, _vp, _vp]),
    "ann_autotune": (_i32, [_vp, _vp, _i64, _i32, _i32, _vp, _vp, C.POINTER(SearchParams), _vp]),
    "ann_server_create": (_i32, [_vp, C.POINTER(ServerParams), C.POINTER(_vp)]),
    "ann_server_footprint": (_i32, [_vp, _i32, _i32, _i32, C.POINTER(_i64), C.POINTER(_i64)]),
    "ann_server_submit": (_i32, [_vp, _vp, _i32, _i32, _i32, C.POINTER(_i64)]),
    "ann_server_progress": (_i32, [_vp, _vp, _i32, C.POINTER(_i32)]),
    "ann_server_result": (_i32, [_vp, _i64, _vp, _vp]),
    "ann_server_drain": (_i32, [_vp]),
    "ann_server_get_info": (_i32, [_vp, C.POINTER(ServerInfo)]),
    "ann_server_destroy": (None, [_vp]),
    "ann_ivf_build": (_i32, [_vp, _i64, _i32, C.POINTER(IvfParams), C.POINTER(_vp)]),
    "ann_ivf_get_info": (_i32, [_vp, C.POINTER(IvfInfo)]),
    "ann_ivf_centres": (_vp, [_vp]),
    "ann_ivf_export": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "ann_ivf_search_device": (_i32, [_vp, _vp, _i64, _i32, _i32, _i32, _i32, _vp, _vp, _vp]),
    "ann_ivf_free": (None, [_vp]),
    "ann_query_tables_device": (_i32, [_vp, _vp, _i64, _vp, _vp, _vp]),
    "ann_knn_device": (_i32, [_vp, _i64, _i32, _i32, _vp, _i64, _i32, _i32, _vp, _vp, _vp]),
    "ann_last_error": (_cp, []),
    "ann_version": (_i32, []),
}


def lib():
    """Load libann.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1312_3062_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != ANN_OK:
        raise AnnError(status, lib().ann_last_error().decode())
