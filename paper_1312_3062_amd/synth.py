"""Seeded synthetic workloads shaped like the paper's SIFT / GIST / HOG sets.

The paper measures on 1M SIFT (128-d bytes), 1M GIST (384-d) and 10M HOG
vectors (Sec. 5.1, "Setup").  None of those sets is available here, so every
workload is a Gaussian mixture drawn from numpy's PCG64 with a fixed seed.
This module holds no arithmetic of the search method itself: it only draws
vectors, queries, per-query budgets and request streams.  Both the oracle
and the HIP path consume what it returns.

Recipe (u8 workloads):
  centres  = U(0, 128)^(C x d) in float64, drawn first from the data stream;
  per chunk of 2^20 rows: labels = integers(0, C), noise = 20 * N(0, 1),
  x = clip(rint(centres[labels] + noise), 0, 255) as uint8.
Queries use the same centres with their own stream.

Recipe (f32, GIST-like): centres U(0, 1)^(C x d), std 0.25, absolute value,
then each row L2-normalised in float64 and stored as float32.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

CHUNK = 1 << 20


@dataclass(frozen=True)
class Workload:
    name: str
    n: int                 # reference vectors
    d: int                 # dimension
    dtype: str             # "u8" or "f32"
    components: int        # mixture components
    nq: int                # queries
    graph_k: int           # R, out-degree of the kNN graph
    P: int                 # subspaces
    K: int                 # codewords per subspace
    k: int                 # neighbours returned
    budgets: tuple         # distance-evaluation budgets T
    queue_len: int = 64    # bound L of the main queue
    bridge_t: int = 1      # nearest bridges kept per reference vector
    bridge_b: int = 0      # reference vectors kept per bridge (0 = all)
    kmeans_iters: int = 10
    seed_base: int = 0     # data = 1000+, queries = 2000+, k-means = 3000+
    center_scale: float = 128.0
    noise_std: float = 20.0
    variable_kT: bool = False   # per-query k in {1,10,100}, T log-uniform

    @property
    def data_seed(self) -> int:
        return 1000 + self.seed_base

    @property
    def query_seed(self) -> int:
        return 2000 + self.seed_base

    @property
    def kmeans_seed(self) -> int:
        return 3000 + self.seed_base

    @property
    def stream_seed(self) -> int:
        return 4000 + self.seed_base


WORKLOADS = {
    # 10K x 128 u8, 64 components; R=10, P=2 x 64 dims, K=32 (1,024 bridges);
    # every reference linked from its nearest bridge; k=10, T=256, L=64.
    "tiny_10k_u8": Workload("tiny_10k_u8", 10_000, 128, "u8", 64, 100, 10, 2, 32, 10,
                            (256,), bridge_t=1, bridge_b=0, seed_base=1),
    # 1M x 128 u8, 256 components; R=16, P=4 x 32 dims, K=32 (1,048,576
    # bridges); t=100, b=5 as in the paper's bridge-graph construction.
    "sift_like_1m_u8": Workload("sift_like_1m_u8", 1_000_000, 128, "u8", 256, 10_000, 16, 4, 32,
                                10, (128, 256, 512, 1024, 2048, 4096, 8192, 16384),
                                bridge_t=100, bridge_b=5, seed_base=2),
    # 1M x 384 f32 GIST-like; R=16, P=3 x 128 dims, K=100 (10^6 bridges).
    "gist_like_1m_f32": Workload("gist_like_1m_f32", 1_000_000, 384, "f32", 128, 1_000, 16, 3,
                                 100, 10, (1024,), bridge_t=100, bridge_b=5, seed_base=3,
                                 center_scale=1.0, noise_std=0.25),
    # 10M x 128 u8 HOG-like; R=16, P=4 x 32, K=64 (16,777,216 bridges);
    # 100K queries with per-query T log-uniform in [64, 4096], k in {1,10,100}.
    "hog_like_10m_u8": Workload("hog_like_10m_u8", 10_000_000, 128, "u8", 1024, 100_000, 16, 4,
                                64, 100, (4096,), bridge_t=100, bridge_b=5, seed_base=4,
                                variable_kT=True),
}


def scaled(w: Workload, n: int, nq: Optional[int] = None, **kw) -> Workload:
    """The same recipe at a smaller size (tests); other fields may be overridden."""
    fields = dict(w.__dict__)
    fields.update(n=n, nq=w.nq if nq is None else nq, name=f"{w.name}@{n}")
    fields.update(kw)
    return Workload(**fields)


def _centres(rng: np.random.Generator, w: Workload) -> np.ndarray:
    return rng.uniform(0.0, w.center_scale, size=(w.components, w.d))


def _draw_rows(rng: np.random.Generator, centres: np.ndarray, m: int, w: Workload) -> np.ndarray:
    labels = rng.integers(0, w.components, size=m)
    x = centres[labels] + w.noise_std * rng.standard_normal((m, w.d))
    if w.dtype == "u8":
        return np.clip(np.rint(x), 0, 255).astype(np.uint8)
    x = np.abs(x)
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x.astype(np.float32)


def _draw(rng: np.random.Generator, centres: np.ndarray, m: int, w: Workload) -> np.ndarray:
    out = np.empty((m, w.d), dtype=np.uint8 if w.dtype == "u8" else np.float32)
    for s in range(0, m, CHUNK):
        e = min(m, s + CHUNK)
        out[s:e] = _draw_rows(rng, centres, e - s, w)
    return out


def base_vectors(w: Workload) -> np.ndarray:
    """The N x d reference set X."""
    rng = np.random.default_rng(w.data_seed)
    centres = _centres(rng, w)
    return _draw(rng, centres, w.n, w)


def queries(w: Workload, nq: Optional[int] = None) -> np.ndarray:
    """nq query vectors drawn around the same centres as X."""
    rng_c = np.random.default_rng(w.data_seed)
    centres = _centres(rng_c, w)
    rng = np.random.default_rng(w.query_seed)
    return _draw(rng, centres, w.nq if nq is None else nq, w)


def per_query_k_budget(w: Workload, nq: Optional[int] = None, lo: int = 64, hi: int = 4096):
    """Uneven batch: k uniform in {1, 10, 100}, T = round(exp(U(ln lo, ln hi)))."""
    m = w.nq if nq is None else nq
    rng = np.random.default_rng(w.stream_seed)
    ks = rng.choice(np.array([1, 10, 100], dtype=np.int32), size=m)
    ts = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=m))).astype(np.int32)
    return ks.astype(np.int32), ts


@dataclass
class Request:
    arrival_s: float
    first: int      # index of the first query vector of the request
    batch: int
    k: int
    budget: int


def request_stream(w: Workload, total_queries: int, rate_rps: float, seed_offset: int = 0,
                   max_batch: int = 1024) -> list:
    """Poisson arrivals; batch = floor(exp(U(0, ln(max_batch+1)))), k in {1,10,100},
    budget uniform over the powers of two 128..8192.  Requests draw consecutive
    query vectors until total_queries are used."""
    rng = np.random.default_rng(w.stream_seed + 17 + seed_offset)
    out, used, clock = [], 0, 0.0
    budgets = np.array([128 << i for i in range(7)], dtype=np.int32)
    while used < total_queries:
        clock += rng.exponential(1.0 / rate_rps)
        b = int(np.floor(np.exp(rng.uniform(0.0, np.log(max_batch + 1)))))
        b = max(1, min(b, max_batch, total_queries - used))
        out.append(Request(clock, used, b, int(rng.choice([1, 10, 100])), int(rng.choice(budgets))))
        used += b
    return out


def graph_seeds(w: Workload, count: int = 16) -> np.ndarray:
    """Fixed seed vectors of the neighborhood-graph search without bridges:
    `count` distinct reference ids drawn once (the same for every query)."""
    rng = np.random.default_rng(5000 + w.seed_base)
    return rng.choice(w.n, size=min(count, w.n), replace=False).astype(np.int32)
