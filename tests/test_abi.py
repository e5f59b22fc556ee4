"""Host-side checks of the C ABI: the library loads, exports every symbol that
include/ann.h declares, and rejects bad arguments before touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1312_3062_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ann.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ann_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("ann_build_index", "ann_search", "ann_search_device", "ann_index_import", "ann_index_export",
                 "ann_index_save", "ann_index_load", "ann_index_free", "ann_last_error", "ann_knn_device",
                 "ann_query_tables_device"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = C.CDLL(_abi.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert set(declared_functions()) <= set(_abi.SIGNATURES)


def test_version_and_error_string():
    L = _abi.lib()
    assert L.ann_version() == 10000
    assert isinstance(L.ann_last_error(), bytes)


def _bp(**kw):
    p = dict(graph_k=4, P=2, K=4, kmeans_iters=2, bridge_t=1, bridge_b=0, reserved=0, seed=1)
    p.update(kw)
    return _abi.BuildParams(C.sizeof(_abi.BuildParams), p["graph_k"], p["P"], p["K"], p["kmeans_iters"],
                            p["bridge_t"], p["bridge_b"], p["reserved"], p["seed"])


@pytest.mark.parametrize("kw,n,d,dtype,msg", [
    (dict(), 0, 16, 0, "n must be"),
    (dict(P=3), 100, 16, 0, "P must divide d"),
    (dict(P=5), 100, 20, 0, "P must be in"),
    (dict(K=0), 100, 16, 0, "K must be in"),
    (dict(K=257), 100, 16, 0, "K must be in"),
    (dict(), 100, 12, 0, "multiple of 16"),
    (dict(), 100, 16, 7, "dtype"),
    (dict(bridge_t=0), 100, 16, 0, "bridge_t"),
    (dict(bridge_b=-1), 100, 16, 0, "bridge_b"),
    (dict(graph_k=100), 100, 16, 0, "graph_k"),
    (dict(reserved=3), 100, 16, 0, "reserved"),
    (dict(K=256, P=4), 100, 16, 0, "2^32"),
    (dict(K=64), 10, 16, 0, "K must not exceed n"),
])
def test_build_rejects_bad_arguments(kw, n, d, dtype, msg):
    L = _abi.lib()
    data = np.zeros((max(n, 1), d), np.uint8)
    h = C.c_void_p()
    bp = _bp(**kw)
    st = L.ann_build_index(data.ctypes.data_as(C.c_void_p), n, d, dtype, C.byref(bp), None, None, C.byref(h))
    assert st == _abi.ANN_EINVAL
    assert msg in L.ann_last_error().decode()
    assert not h.value


def test_build_rejects_null_and_struct_size():
    L = _abi.lib()
    h = C.c_void_p()
    bp = _bp()
    assert L.ann_build_index(None, 10, 16, 0, C.byref(bp), None, None, C.byref(h)) == _abi.ANN_EINVAL
    bad = _bp()
    bad.struct_size = 7
    data = np.zeros((10, 16), np.uint8)
    assert L.ann_build_index(data.ctypes.data_as(C.c_void_p), 10, 16, 0, C.byref(bad), None, None,
                             C.byref(h)) == _abi.ANN_EINVAL
    assert "struct_size" in L.ann_last_error().decode()


def test_build_rejects_bad_graph_rows():
    L = _abi.lib()
    data = np.zeros((10, 16), np.uint8)
    g = np.zeros((10, 2), np.uint32)   # repeats id 0 in every row
    bp = _bp(graph_k=2)
    h = C.c_void_p()
    st = L.ann_build_index(data.ctypes.data_as(C.c_void_p), 10, 16, 0, C.byref(bp), None,
                           g.ctypes.data_as(C.c_void_p), C.byref(h))
    assert st == _abi.ANN_EINVAL and "repeats" in L.ann_last_error().decode()
    g2 = np.full((10, 2), 99, np.uint32)
    st = L.ann_build_index(data.ctypes.data_as(C.c_void_p), 10, 16, 0, C.byref(bp), None,
                           g2.ctypes.data_as(C.c_void_p), C.byref(h))
    assert st == _abi.ANN_EINVAL and "out of range" in L.ann_last_error().decode()


def test_import_rejects_inconsistent_parts():
    L = _abi.lib()
    X = np.zeros((6, 16), np.uint8)
    cb = np.zeros((2, 2, 8), np.uint8)
    off = np.array([0, 2, 2, 3, 3], np.uint32)
    ids = np.array([0, 0, 1], np.uint32)    # list 0 repeats id 0
    h = C.c_void_p()
    p = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
    st = L.ann_index_import(p(X), 6, 16, 0, 2, 2, p(cb), 0, None, p(off), p(ids), C.byref(h))
    assert st == _abi.ANN_EINVAL and "repeats" in L.ann_last_error().decode()
    off2 = np.array([0, 2, 1, 3, 3], np.uint32)
    ids2 = np.array([0, 1, 2], np.uint32)
    st = L.ann_index_import(p(X), 6, 16, 0, 2, 2, p(cb), 0, None, p(off2), p(ids2), C.byref(h))
    assert st == _abi.ANN_EINVAL and "non-decreasing" in L.ann_last_error().decode()
    ids3 = np.array([0, 1, 9], np.uint32)
    st = L.ann_index_import(p(X), 6, 16, 0, 2, 2, p(cb), 0, None, p(off), p(ids3), C.byref(h))
    assert st == _abi.ANN_EINVAL and "out of range" in L.ann_last_error().decode()


def test_search_rejects_bad_arguments_without_an_index():
    L = _abi.lib()
    sp = _abi.SearchParams(C.sizeof(_abi.SearchParams), 64, 0, 0)
    st = L.ann_search_device(None, None, 1, 10, 10, None, None, C.byref(sp), None, None, None, None, None)
    assert st == _abi.ANN_EINVAL and "null index" in L.ann_last_error().decode()


def test_load_rejects_missing_and_foreign_files(tmp_path):
    L = _abi.lib()
    h = C.c_void_p()
    assert L.ann_index_load(str(tmp_path / "nope.bin").encode(), C.byref(h)) == _abi.ANN_EIO
    f = tmp_path / "junk.bin"
    f.write_bytes(b"not an index at all, definitely not")
    assert L.ann_index_load(str(f).encode(), C.byref(h)) == _abi.ANN_EIO
