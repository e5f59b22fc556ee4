"""Request serving over a device-resident index: continuous batching vs plain launches.

Served: requests (a batch of query vectors with its own k and budget) arrive
on a clock and are handed to the library's request server (ann_server_* in
include/ann.h).  The server admits pending requests into micro-batches by
their device-memory and LDS footprint whenever a launch slot is free; slots
run on their own streams, so requests that arrive while others are on the
GPU are admitted as slots and memory free up and their work overlaps on the
device.  This module only simulates the arrivals and collects completions.

Plain: each request is launched on its own, in arrival order, on one stream,
and waits for the previous one to finish.

Latency of a request = completion time - arrival time (host monotonic clock;
completion is when the host sees the request's micro-batch finished).
Results of a query are the same in both modes and in any mix: the search of
a query depends only on (index, query, k, budget, queue length).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class RunResult:
    mode: str
    rate_rps: float
    requests: int
    queries: int
    wall_s: float
    latencies_s: np.ndarray
    ids: Optional[np.ndarray] = None           # per query, padded to max k
    launches: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def qps(self) -> float:
        return self.queries / self.wall_s if self.wall_s > 0 else 0.0

    def summary(self) -> dict:
        lat = self.latencies_s * 1e3
        return {"mode": self.mode, "rate_rps": round(self.rate_rps, 2), "requests": self.requests,
                "queries": self.queries, "wall_s": round(self.wall_s, 4), "qps": round(self.qps, 1),
                "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "mean_ms": round(float(lat.mean()), 3), "launches": self.launches, **self.extra}


class _Slot:
    """Buffers of the plain (one launch per request) baseline."""

    def __init__(self, torch, d: int, cap: int, kmax: int, qdtype):
        self.stream = torch.cuda.Stream()          # default priority
        self.q_host = torch.empty((cap, d), dtype=qdtype, pin_memory=True)
        self.q_dev = torch.empty((cap, d), dtype=qdtype, device="cuda")
        self.ids_host = torch.empty((cap, kmax), dtype=torch.int32, pin_memory=True)
        self.d_host = torch.empty((cap, kmax), dtype=torch.int32 if qdtype == torch.uint8 else torch.float32,
                                  pin_memory=True)
        self.done = torch.cuda.Event()


class Server:
    """Continuous batching through the library's request server (ann_server_*)."""

    def __init__(self, index, d: int, qdtype="u8", slots: int = 4, slot_queries: int = 4096, kmax: int = 100,
                 max_budget: int = 8192, queue_len: int = 64, tune: Optional[dict] = None, device_bytes: int = 0,
                 lds_rounds: int = 0):
        import ctypes as C

        import torch

        from . import _abi
        from .index import search_params
        self.torch = torch
        self.C = C
        self._abi = _abi
        self.index = index
        self.kmax = kmax
        self.max_budget = max_budget
        self.queue_len = queue_len
        self.qdtype = np.uint8 if qdtype == "u8" else np.float32
        self.tune = tune if tune is not None else {}
        self.slot_queries = slot_queries
        sp = search_params(queue_len, 0, 0, self.tune)
        p = _abi.ServerParams(C.sizeof(_abi.ServerParams), slots, slot_queries, kmax, max_budget, lds_rounds,
                              device_bytes, sp)
        h = C.c_void_p()
        _abi.check(_abi.lib().ann_server_create(index._h, C.byref(p), C.byref(h)))
        self._h = h
        self._plain = _Slot(torch, d, slot_queries, kmax, torch.uint8 if qdtype == "u8" else torch.float32)

    def close(self):
        if getattr(self, "_h", None):
            self._abi.lib().ann_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        inf = self._abi.ServerInfo()
        self._abi.check(self._abi.lib().ann_server_get_info(self._h, self.C.byref(inf)))
        return {f: getattr(inf, f) for f, _ in self._abi.ServerInfo._fields_}

    def footprint(self, nq: int, k: int, budget: int) -> dict:
        lds, dev = self.C.c_int64(), self.C.c_int64()
        self._abi.check(self._abi.lib().ann_server_footprint(self._h, nq, k, budget, self.C.byref(lds),
                                                             self.C.byref(dev)))
        return {"lds_bytes": lds.value, "device_bytes": dev.value}

    # ---------------------------------------------------------------- served
    def run_served(self, requests, pool: np.ndarray, rate_rps: float = 0.0, keep_ids: bool = False) -> RunResult:
        C, L, check = self.C, self._abi.lib(), self._abi.check
        pool = np.ascontiguousarray(pool, dtype=self.qdtype)
        arrivals = np.array([r.arrival_s for r in requests])
        lat = np.zeros(len(requests))
        offs = np.cumsum([0] + [r.batch for r in requests])
        ids_out = np.full((int(offs[-1]), self.kmax), -1, np.int32) if keep_ids else None
        ids_buf = np.empty(self.slot_queries * self.kmax, np.int32)
        d_buf = np.empty(self.slot_queries * self.kmax, np.int32 if self.qdtype == np.uint8 else np.float32)
        done = (C.c_int64 * 4096)()
        n_done = C.c_int32()
        ticket = C.c_int64()
        launches0 = self.info()["launches"]
        by_ticket = {}
        nxt = finished = 0
        t0 = time.perf_counter()
        while finished < len(requests):
            now = time.perf_counter() - t0
            while nxt < len(requests) and arrivals[nxt] <= now:
                r = requests[nxt]
                q = pool[r.first:r.first + r.batch]
                check(L.ann_server_submit(self._h, q.ctypes.data_as(C.c_void_p), r.batch, r.k, r.budget,
                                          C.byref(ticket)))
                by_ticket[ticket.value] = nxt
                nxt += 1
            check(L.ann_server_progress(self._h, done, len(done), C.byref(n_done)))
            if n_done.value:
                tdone = time.perf_counter() - t0
                for t in done[:n_done.value]:
                    ri = by_ticket.pop(t)
                    r = requests[ri]
                    check(L.ann_server_result(self._h, t, ids_buf.ctypes.data_as(C.c_void_p),
                                              d_buf.ctypes.data_as(C.c_void_p)))
                    if keep_ids:
                        ids_out[offs[ri]:offs[ri] + r.batch, :r.k] = ids_buf[:r.batch * r.k].reshape(r.batch, r.k)
                    lat[ri] = tdone - arrivals[ri]
                    finished += 1
            elif nxt < len(requests) and not by_ticket:
                # idle: wait for the next arrival
                wait = arrivals[nxt] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.001))
        wall = time.perf_counter() - t0 - float(arrivals[0] if len(arrivals) else 0.0)
        launches = self.info()["launches"] - launches0
        return RunResult("served", rate_rps, len(requests), int(offs[-1]), wall, lat, ids_out, launches)

    # ---------------------------------------------------------------- plain
    def run_plain(self, requests, pool: np.ndarray, rate_rps: float = 0.0, keep_ids: bool = False) -> RunResult:
        """One launch per request, in arrival order, on one stream."""
        torch = self.torch
        sl = self._plain
        arrivals = np.array([r.arrival_s for r in requests])
        lat = np.zeros(len(requests))
        offs = np.cumsum([0] + [r.batch for r in requests])
        ids_out = np.full((int(offs[-1]), self.kmax), -1, np.int32) if keep_ids else None
        t0 = time.perf_counter()
        for ri, r in enumerate(requests):
            wait = arrivals[ri] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            qh = sl.q_host.numpy()
            qh[:r.batch] = pool[r.first:r.first + r.batch]
            with torch.cuda.stream(sl.stream):
                sl.q_dev[:r.batch].copy_(sl.q_host[:r.batch], non_blocking=True)
                ids, dd = self.index.search_device(sl.q_dev[:r.batch], r.k, r.budget, queue_len=self.queue_len,
                                                   stream=sl.stream)
                # results come back to the host, as the server's do
                sl.ids_host[:r.batch, :r.k].copy_(ids, non_blocking=True)
                sl.d_host[:r.batch, :r.k].copy_(dd, non_blocking=True)
                sl.done.record(sl.stream)
            sl.done.synchronize()
            lat[ri] = time.perf_counter() - t0 - arrivals[ri]
            if keep_ids:
                ids_out[offs[ri]:offs[ri] + r.batch, :r.k] = sl.ids_host.numpy()[:r.batch, :r.k]
        wall = time.perf_counter() - t0 - float(arrivals[0] if len(arrivals) else 0.0)
        return RunResult("plain", rate_rps, len(requests), int(offs[-1]), wall, lat, ids_out, len(requests))

    def plain_service_time(self, requests, pool: np.ndarray) -> float:
        """Mean time of one plain launch per request (back to back): 1 / saturation rate."""
        import copy
        rs = [copy.copy(r) for r in requests]
        for r in rs:
            r.arrival_s = 0.0
        res = self.run_plain(rs, pool)
        return res.wall_s / max(1, len(rs))
