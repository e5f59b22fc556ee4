"""Python binding of the HIP library: argument marshalling around include/ann.h.

Every step of the search and of the index build runs in the library's HIP
kernels.  PyTorch only provides device memory and the current stream.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import _abi
from ._abi import check, lib

_DT = {np.dtype(np.uint8): _abi.ANN_U8, np.dtype(np.float32): _abi.ANN_F32}


def _np_ptr(a: Optional[np.ndarray]):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _dtype_code(a) -> int:
    dt = np.dtype(a.dtype) if isinstance(a, np.ndarray) else _torch_np_dtype(a)
    if dt not in _DT:
        raise TypeError(f"unsupported dtype {dt}: use uint8 or float32")
    return _DT[dt]


def _torch_np_dtype(t):
    import torch
    return {torch.uint8: np.dtype(np.uint8), torch.float32: np.dtype(np.float32)}.get(t.dtype, None)


def _tptr(t) -> Optional[C.c_void_p]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _stream_ptr(stream=None) -> Optional[C.c_void_p]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


TUNING_KEYS = ("lookahead", "persistent", "waves_per_cu", "order")


def search_params(queue_len: int = 64, precision: int = 0, rerank_k: int = 0, tune: Optional[dict] = None
                  ) -> _abi.SearchParams:
    """ann_search_params; `tune` holds launch-tuning fields (results never depend on them)."""
    t = tune or {}
    return _abi.SearchParams(C.sizeof(_abi.SearchParams), queue_len, precision, rerank_k,
                             *(int(t.get(key, 0)) for key in TUNING_KEYS))


class Index:
    """Owns an ann_index handle (device-resident index)."""

    def __init__(self, handle: C.c_void_p):
        self._h = handle

    # ---- construction
    @classmethod
    def build(cls, data: np.ndarray, graph_k: int, P: int, K: int, kmeans_iters: int = 10, seed: int = 0,
              bridge_t: int = 1, bridge_b: int = 0, codebooks: Optional[np.ndarray] = None,
              graph: Optional[np.ndarray] = None) -> "Index":
        data = np.ascontiguousarray(data)
        n, d = data.shape
        bp = _abi.BuildParams(C.sizeof(_abi.BuildParams), graph_k, P, K, kmeans_iters, bridge_t, bridge_b, 0, seed)
        cb = None if codebooks is None else np.ascontiguousarray(codebooks, dtype=data.dtype)
        g = None if graph is None else np.ascontiguousarray(graph, dtype=np.uint32)
        h = C.c_void_p()
        check(lib().ann_build_index(_np_ptr(data), n, d, _dtype_code(data), C.byref(bp), _np_ptr(cb), _np_ptr(g),
                                    C.byref(h)))
        return cls(h)

    @classmethod
    def from_parts(cls, data: np.ndarray, codebooks: np.ndarray, graph: Optional[np.ndarray], bridge_off: np.ndarray,
                   bridge_ids: np.ndarray) -> "Index":
        data = np.ascontiguousarray(data)
        n, d = data.shape
        P, K, _ = codebooks.shape
        cb = np.ascontiguousarray(codebooks, dtype=data.dtype)
        R = 0 if graph is None or graph.size == 0 else graph.shape[1]
        g = None if R == 0 else np.ascontiguousarray(graph, dtype=np.uint32)
        off = np.ascontiguousarray(bridge_off, dtype=np.uint32)
        ids = np.ascontiguousarray(bridge_ids, dtype=np.uint32)
        if ids.size == 0:
            ids = np.zeros(1, np.uint32)
        h = C.c_void_p()
        check(lib().ann_index_import(_np_ptr(data), n, d, _dtype_code(data), P, K, _np_ptr(cb), R, _np_ptr(g),
                                     _np_ptr(off), _np_ptr(ids), C.byref(h)))
        return cls(h)

    @classmethod
    def load(cls, path: str) -> "Index":
        h = C.c_void_p()
        check(lib().ann_index_load(path.encode(), C.byref(h)))
        return cls(h)

    def save(self, path: str) -> None:
        check(lib().ann_index_save(self._h, path.encode()))

    def close(self) -> None:
        if self._h:
            lib().ann_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- inspection
    @property
    def info(self) -> dict:
        inf = _abi.IndexInfo()
        check(lib().ann_index_get_info(self._h, C.byref(inf)))
        return {f: getattr(inf, f) for f, _ in _abi.IndexInfo._fields_}

    def export(self) -> dict:
        inf = self.info
        dt = np.uint8 if inf["dtype"] == _abi.ANN_U8 else np.float32
        P, K, d = inf["P"], inf["K"], inf["d"]
        cb = np.empty((P, K, d // P), dt)
        g = np.empty((inf["n"], inf["graph_k"]), np.uint32)
        off = np.empty(inf["n_bridges"] + 1, np.uint32)
        ids = np.empty(max(1, inf["n_bridge_entries"]), np.uint32)
        check(lib().ann_index_export(self._h, _np_ptr(cb), _np_ptr(g) if g.size else None, _np_ptr(off),
                                     _np_ptr(ids)))
        return {"codebooks": cb, "graph": g, "bridge_off": off, "bridge_ids": ids[:inf["n_bridge_entries"]]}

    # ---- search
    def search(self, queries: np.ndarray, k: int, budget: int, queue_len: int = 64, precision: int = 0,
               rerank_k: int = 0):
        """Host-buffer search; returns (ids int32, dists int32|float32), both nq x k."""
        q = np.ascontiguousarray(queries)
        nq = q.shape[0]
        ids = np.empty((nq, k), np.int32)
        dists = np.empty((nq, k), np.int32 if q.dtype == np.uint8 else np.float32)
        sp = search_params(queue_len, precision, rerank_k)
        check(lib().ann_search(self._h, _np_ptr(q), nq, k, budget, C.byref(sp), _np_ptr(ids), _np_ptr(dists)))
        return ids, dists

    def search_device(self, queries, k: int, budget: int, ks=None, budgets=None, queue_len: int = 64,
                      precision: int = 0, rerank_k: int = 0, out=None, stats=None, trace=None, stream=None,
                      tune: Optional[dict] = None, workspace=None):
        """Device search on torch tensors, asynchronous on `stream` (default: current).

        Returns (ids, dists) tensors of shape nq x k.  `stats` (nq x 12 int32) and
        `trace` (nq x budget int32) are optional output tensors.  `tune` holds
        launch settings (see TUNING_KEYS).  With `workspace` (a uint8 device
        tensor of at least workspace_bytes(...)) the call allocates nothing."""
        import torch
        nq = queries.shape[0]
        dev = queries.device
        if out is None:
            ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
            dd = torch.empty((nq, k), dtype=torch.int32 if queries.dtype == torch.uint8 else torch.float32,
                             device=dev)
        else:
            ids, dd = out
        sp = search_params(queue_len, precision, rerank_k, tune)
        if workspace is None:
            check(lib().ann_search_device(self._h, _tptr(queries), nq, k, budget, _tptr(ks), _tptr(budgets),
                                          C.byref(sp), _tptr(ids), _tptr(dd), _tptr(stats), _tptr(trace),
                                          _stream_ptr(stream)))
        else:
            check(lib().ann_search_device_ws(self._h, _tptr(queries), nq, k, budget, _tptr(ks), _tptr(budgets),
                                             C.byref(sp), _tptr(ids), _tptr(dd), _tptr(stats), _tptr(trace),
                                             _tptr(workspace), workspace.numel(), _stream_ptr(stream)))
        return ids, dd

    def search_graph_device(self, queries, k: int, budget: int, seeds, queue_len: int = 64, out=None, stats=None,
                            trace=None, stream=None, tune: Optional[dict] = None):
        """Neighborhood-graph search without bridges (Sec. 2.2): `seeds` (int32
        device tensor of reference ids) are measured first, then the kNN graph
        is expanded best first.  Returns (ids, dists) tensors nq x k."""
        import torch
        nq = queries.shape[0]
        dev = queries.device
        if out is None:
            ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
            dd = torch.empty((nq, k), dtype=torch.int32 if queries.dtype == torch.uint8 else torch.float32,
                             device=dev)
        else:
            ids, dd = out
        sp = search_params(queue_len, 0, 0, tune)
        check(lib().ann_search_graph_device(self._h, _tptr(queries), nq, k, budget, _tptr(seeds), seeds.numel(),
                                            C.byref(sp), _tptr(ids), _tptr(dd), _tptr(stats), _tptr(trace),
                                            _stream_ptr(stream)))
        return ids, dd

    def workspace_bytes(self, nq: int, k: int, budget: int, queue_len: int = 64, precision: int = 0,
                        rerank_k: int = 0, tune: Optional[dict] = None) -> int:
        sp = search_params(queue_len, precision, rerank_k, tune)
        out = C.c_int64()
        check(lib().ann_search_workspace_size(self._h, nq, k, budget, C.byref(sp), C.byref(out)))
        return out.value

    def autotune(self, queries, k: int, budget: int, ks=None, budgets=None, queue_len: int = 64,
                 precision: int = 0, rerank_k: int = 0, stream=None) -> dict:
        """Time the launch settings on this batch; returns the fastest as a `tune` dict."""
        sp = search_params(queue_len, precision, rerank_k)
        check(lib().ann_autotune(self._h, _tptr(queries), queries.shape[0], k, budget, _tptr(ks), _tptr(budgets),
                                 C.byref(sp), _stream_ptr(stream)))
        return {key: getattr(sp, key) for key in TUNING_KEYS}

    def tables_device(self, queries, stream=None):
        """(sorted values, codeword of each rank) per query, shapes nq x P x K."""
        import torch
        inf = self.info
        nq = queries.shape[0]
        vt = torch.int32 if inf["dtype"] == _abi.ANN_U8 else torch.float32
        sv = torch.empty((nq, inf["P"], inf["K"]), dtype=vt, device=queries.device)
        perm = torch.empty((nq, inf["P"], inf["K"]), dtype=torch.int32, device=queries.device)
        check(lib().ann_query_tables_device(self._h, _tptr(queries), nq, _tptr(sv), _tptr(perm),
                                            _stream_ptr(stream)))
        return sv, perm


def knn_device(x, q, k: int, exclude_self: bool = False, stream=None):
    """Exact kNN by linear scan on device tensors; returns (ids, dists) nq x k."""
    import torch
    n, d = x.shape
    nq = q.shape[0]
    ids = torch.empty((nq, k), dtype=torch.int32, device=x.device)
    dd = torch.empty((nq, k), dtype=torch.int32 if x.dtype == torch.uint8 else torch.float32, device=x.device)
    check(lib().ann_knn_device(_tptr(x), n, d, _dtype_code(x), _tptr(q), nq, k, int(exclude_self), _tptr(ids),
                               _tptr(dd), _stream_ptr(stream)))
    return ids, dd


def recall_at(found: np.ndarray, truth: np.ndarray, k: int) -> float:
    """Mean over queries of |found[:k] & truth[:k]| / k (the paper's accuracy r/k, Sec. 5.1)."""
    f = np.asarray(found)[:, :k]
    t = np.asarray(truth)[:, :k]
    hits = 0
    for a, b in zip(f, t):
        hits += len(set(a[a >= 0].tolist()) & set(b[b >= 0].tolist()))
    return hits / (k * len(f)) if len(f) else 0.0
