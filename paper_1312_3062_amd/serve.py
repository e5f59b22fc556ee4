"""Request serving over a device-resident index: continuous batching vs plain launches.

Served: requests (a batch of query vectors with its own k and budget) arrive
on a clock.  Whenever a launch slot is free, every request that has arrived
and fits the slot's footprint is admitted into one micro-batch: its queries
are copied to the device and searched by one launch with per-query k and
budget, on the slot's own stream.  Several slots are in flight at once, so
requests that arrive while others are on the GPU are admitted as soon as a
slot frees up and their work overlaps on the device.

Plain: each request is launched on its own, in arrival order, on one stream,
and waits for the previous one to finish.

Latency of a request = completion time - arrival time (host monotonic clock).
Results of a query are the same in both modes and in any mix: the search of a
query depends only on (index, query, k, budget, queue length).
"""
from __future__ import annotations

import collections
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
    def __init__(self, torch, d: int, cap: int, kmax: int, qdtype):
        self.stream = torch.cuda.Stream()          # default priority
        self.q_host = torch.empty((cap, d), dtype=qdtype, pin_memory=True)
        self.kt_host = torch.empty((2, cap), dtype=torch.int32, pin_memory=True)
        self.q_dev = torch.empty((cap, d), dtype=qdtype, device="cuda")
        self.kt_dev = torch.empty((2, cap), dtype=torch.int32, device="cuda")
        self.ids = torch.empty((cap, kmax), dtype=torch.int32, device="cuda")
        self.dd = torch.empty((cap, kmax), dtype=torch.int32 if qdtype == torch.uint8 else torch.float32,
                              device="cuda")
        self.ids_host = torch.empty((cap, kmax), dtype=torch.int32, pin_memory=True)
        self.done = torch.cuda.Event()
        self.reqs = []
        self.groups = []
        self.busy = False


class Server:
    """Continuous-batching request loop over an Index (device-resident)."""

    def __init__(self, index, d: int, qdtype="u8", slots: int = 4, slot_queries: int = 4096, kmax: int = 100,
                 queue_len: int = 64, tune: Optional[dict] = None, footprint_queries: Optional[int] = None):
        import torch
        self.torch = torch
        self.index = index
        self.kmax = kmax
        self.queue_len = queue_len
        self.tune = tune if tune is not None else {"persistent": 1, "order": 1}
        tq = torch.uint8 if qdtype == "u8" else torch.float32
        self.slots = [_Slot(torch, d, slot_queries, kmax, tq) for _ in range(slots)]
        self.slot_queries = slot_queries
        # admission: queries in flight over all slots (device-memory footprint of outputs and state)
        self.footprint_queries = footprint_queries or slots * slot_queries

    # ---------------------------------------------------------------- served
    def run_served(self, requests, pool: np.ndarray, rate_rps: float = 0.0, keep_ids: bool = False) -> RunResult:
        torch = self.torch
        arrivals = np.array([r.arrival_s for r in requests])
        lat = np.zeros(len(requests))
        ids_out = np.full((sum(r.batch for r in requests), self.kmax), -1, np.int32) if keep_ids else None
        offs = np.cumsum([0] + [r.batch for r in requests])
        pending = collections.deque()
        nxt = 0
        inflight_q = 0
        launches = 0
        t0 = time.perf_counter()
        finished = 0
        while finished < len(requests):
            now = time.perf_counter() - t0
            while nxt < len(requests) and arrivals[nxt] <= now:
                pending.append(nxt)
                nxt += 1
            # completions
            for sl in self.slots:
                if sl.busy and sl.done.query():
                    tdone = time.perf_counter() - t0
                    if keep_ids:
                        sl.stream.synchronize()
                        self._collect_ids(sl, requests, ids_out, offs)
                    for ri in sl.reqs:
                        lat[ri] = tdone - arrivals[ri]
                        inflight_q -= requests[ri].batch
                    finished += len(sl.reqs)
                    sl.reqs = []
                    sl.busy = False
            # admission into a free slot
            free = [sl for sl in self.slots if not sl.busy]
            while pending and free:
                sl = free.pop()
                take, nq = [], 0
                while pending:
                    ri = pending[0]
                    b = requests[ri].batch
                    if nq + b > self.slot_queries or inflight_q + nq + b > self.footprint_queries:
                        break
                    take.append(pending.popleft())
                    nq += b
                if not take:
                    free.append(sl)
                    break
                self._launch(sl, requests, take, nq, pool, keep_ids)
                inflight_q += nq
                launches += 1
            if not pending and nxt < len(requests) and all(not s.busy for s in self.slots):
                # idle: wait for the next arrival
                wait = arrivals[nxt] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.001))
        wall = time.perf_counter() - t0 - float(arrivals[0] if len(arrivals) else 0.0)
        return RunResult("served", rate_rps, len(requests), int(offs[-1]), wall, lat, ids_out, launches)

    # budget classes launched separately inside a micro-batch: per-query LDS is
    # sized by the largest budget of a launch
    CLASS_LIMITS = (512, 2048, 1 << 20)

    def _launch(self, sl: _Slot, requests, take, nq: int, pool: np.ndarray, keep_ids: bool):
        torch = self.torch
        qh = sl.q_host.numpy()
        kt = sl.kt_host.numpy()
        cls = lambda r: next(i for i, lim in enumerate(self.CLASS_LIMITS) if r.budget <= lim)  # noqa: E731
        take = sorted(take, key=lambda ri: cls(requests[ri]))
        row = 0
        groups = []  # (class, first row, end row, kmax, tmax)
        for ri in take:
            r = requests[ri]
            c = cls(r)
            if not groups or groups[-1][0] != c:
                groups.append([c, row, row, 1, 1])
            g = groups[-1]
            qh[row:row + r.batch] = pool[r.first:r.first + r.batch]
            kt[0, row:row + r.batch] = r.k
            kt[1, row:row + r.batch] = r.budget
            row += r.batch
            g[2] = row
            g[3] = max(g[3], r.k)
            g[4] = max(g[4], r.budget)
        ids_flat = sl.ids.view(-1)
        dd_flat = sl.dd.view(-1)
        with torch.cuda.stream(sl.stream):
            sl.q_dev[:nq].copy_(sl.q_host[:nq], non_blocking=True)
            sl.kt_dev[:, :nq].copy_(sl.kt_host[:, :nq], non_blocking=True)
            out_off = 0
            sl.groups = []
            for _, a, b, kmax, tmax in groups:
                m = b - a
                ids = ids_flat[out_off:out_off + m * kmax].view(m, kmax)
                dd = dd_flat[out_off:out_off + m * kmax].view(m, kmax)
                self.index.search_device(sl.q_dev[a:b], kmax, tmax, ks=sl.kt_dev[0, a:b], budgets=sl.kt_dev[1, a:b],
                                         queue_len=self.queue_len, out=(ids, dd), tune=self.tune, stream=sl.stream)
                sl.groups.append((a, b, kmax, out_off))
                out_off += m * kmax
            if keep_ids:
                sl.ids_host.view(-1)[:out_off].copy_(ids_flat[:out_off], non_blocking=True)
            sl.done.record(sl.stream)
        sl.reqs = list(take)
        sl.busy = True

    def _collect_ids(self, sl: _Slot, requests, ids_out: np.ndarray, offs: np.ndarray):
        flat = sl.ids_host.numpy().reshape(-1)
        rows = {}
        for a, b, kmax, o in sl.groups:
            rows.update({a + i: flat[o + i * kmax:o + (i + 1) * kmax] for i in range(b - a)})
        row = 0
        for ri in sl.reqs:
            r = requests[ri]
            for i in range(r.batch):
                v = rows[row + i]
                ids_out[offs[ri] + i, :len(v)] = v
            row += r.batch

    # ---------------------------------------------------------------- plain
    def run_plain(self, requests, pool: np.ndarray, rate_rps: float = 0.0, keep_ids: bool = False) -> RunResult:
        """One launch per request, in arrival order, on one stream."""
        torch = self.torch
        sl = self.slots[0]
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
                if keep_ids:
                    sl.ids_host[:r.batch, :r.k].copy_(ids, non_blocking=True)
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
