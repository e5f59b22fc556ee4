"""Graph-D-ADC (Sec. 5): inverted lists over coarse centres found by the
augmented-graph search, product-quantised residuals and asymmetric-distance
re-ranking.  Argument marshalling for the ann_ivf_* calls of include/ann.h;
every step runs in libann.so."""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import _abi
from ._abi import check, lib
from .index import Index, _np_ptr, _stream_ptr, _tptr


class _CentresView(Index):
    """The centres' index, owned by its Ivf (never freed from here)."""

    def __init__(self, handle, owner):
        super().__init__(handle)
        self._owner = owner

    def close(self) -> None:
        self._h = None


class Ivf:
    """Owns an ann_ivf handle."""

    def __init__(self, handle: C.c_void_p):
        self._h = handle

    @classmethod
    def build(cls, data: np.ndarray, lists: int, pq_m: int, pq_iters: int = 4, assign_budget: int = 256,
              seed: int = 0, graph_k: int = 16, P: int = 2, K: int = 16, kmeans_iters: int = 4, bridge_t: int = 1,
              bridge_b: int = 0, centre_seed: int = 0) -> "Ivf":
        data = np.ascontiguousarray(data, dtype=np.uint8)
        n, d = data.shape
        bp = _abi.BuildParams(C.sizeof(_abi.BuildParams), graph_k, P, K, kmeans_iters, bridge_t, bridge_b, 0,
                              centre_seed)
        ip = _abi.IvfParams(C.sizeof(_abi.IvfParams), lists, pq_m, pq_iters, assign_budget, 0, seed, bp)
        h = C.c_void_p()
        check(lib().ann_ivf_build(_np_ptr(data), n, d, C.byref(ip), C.byref(h)))
        return cls(h)

    def close(self) -> None:
        if self._h:
            lib().ann_ivf_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def info(self) -> dict:
        inf = _abi.IvfInfo()
        check(lib().ann_ivf_get_info(self._h, C.byref(inf)))
        return {f: getattr(inf, f) for f, _ in _abi.IvfInfo._fields_}

    def centres_index(self) -> Index:
        return _CentresView(C.c_void_p(lib().ann_ivf_centres(self._h)), self)

    def export(self) -> dict:
        inf = self.info
        n, d, C_, m = inf["n"], inf["d"], inf["lists"], inf["pq_m"]
        centres = np.empty((C_, d), np.uint8)
        off = np.empty(C_ + 1, np.uint32)
        ids = np.empty(n, np.uint32)
        codes = np.empty((n, m), np.uint8)
        pq = np.empty((m, 256, d // m), np.float32)
        check(lib().ann_ivf_export(self._h, _np_ptr(centres), _np_ptr(off), _np_ptr(ids), _np_ptr(codes),
                                   _np_ptr(pq)))
        return {"centres": centres, "list_off": off, "list_ids": ids, "codes": codes, "pq": pq}

    def search_device(self, queries, k: int, lists: int, centre_budget: int, candidates: int, out=None,
                      stream=None):
        """queries: (nq, d) uint8 device tensor.  Returns (ids int32, dists float32) device tensors (nq, k)."""
        import torch
        nq = queries.shape[0]
        if out is None:
            out = (torch.empty((nq, k), dtype=torch.int32, device=queries.device),
                   torch.empty((nq, k), dtype=torch.float32, device=queries.device))
        ids, dists = out
        check(lib().ann_ivf_search_device(self._h, _tptr(queries), nq, k, lists, centre_budget, candidates,
                                          _tptr(ids), _tptr(dists), _stream_ptr(stream)))
        return ids, dists
