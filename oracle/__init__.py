"""ctypes wrapper around the CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the slow reference the HIP library is checked
against.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
may import this package; the product path never does.  It shares no code
with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

U8, F32 = 0, 1


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (single-threaded C99)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def load(path: str):
    """Open a compiled oracle library and declare its functions."""
    L = C.CDLL(path)
    vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int
    L.orc_knn.argtypes = [vp, i64, i32, i32, vp, i64, vp, i32, vp, vp]
    L.orc_splitmix64.argtypes = [C.c_uint64, i64, vp]
    L.orc_init_rows.argtypes = [i64, i32, C.c_uint64, vp]
    L.orc_kmeans.argtypes = [vp, i64, i32, i32, i32, i32, i32, C.c_uint64, vp, vp]
    L.orc_tables.argtypes = [vp, i32, i32, i32, i32, vp, vp]
    L.orc_sort_tables.argtypes = [i32, i32, vp, vp, vp]
    L.orc_mseq.argtypes = [i32, i32, vp, i64, vp, vp, vp]
    L.orc_mseq.restype = i64
    L.orc_bridge_graph.argtypes = [vp, i64, i32, i32, i32, i32, vp, i32, i32, vp, vp, vp, i64]
    L.orc_bridge_graph.restype = i64
    L.orc_search.argtypes = [vp, i64, i32, i32, i32, i32, vp, i32, vp, vp, vp, vp, i64,
                             vp, vp, i32, i32, vp, vp, vp, i32, vp]
    L.orc_search_ex.argtypes = [vp, i64, i32, i32, i32, i32, vp, i32, vp, vp, vp, vp, i64,
                                vp, vp, i32, i32, i32, i32, i32, vp, i32, vp, vp, vp, i32, vp]
    L.orc_bf16_round.argtypes = [vp, i64, vp]
    L.orc_pq_encode.argtypes = [vp, i64, i32, i32, i32, vp, vp, vp]
    L.orc_ivf_adc.argtypes = [vp, i64, i32, vp, vp, vp, vp, i32, i32, vp, vp, i32, i64, i32, vp, vp, vp]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = load(LIB)
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _dt(x: np.ndarray) -> int:
    if x.dtype == np.uint8:
        return U8
    if x.dtype == np.float32:
        return F32
    raise TypeError(f"unsupported dtype {x.dtype}")


def knn(X: np.ndarray, Q: np.ndarray, k: int, exclude=None):
    """Exact k nearest neighbours of each row of Q in X, ascending by (D, id).
    Returns (ids int32, dists float64)."""
    X = np.ascontiguousarray(X)
    Q = np.ascontiguousarray(Q, dtype=X.dtype)
    nq = Q.shape[0]
    ids = np.empty((nq, k), np.int32)
    d = np.empty((nq, k), np.float64)
    ex = None if exclude is None else np.ascontiguousarray(exclude, dtype=np.int64)
    lib().orc_knn(_p(X), X.shape[0], X.shape[1], _dt(X), _p(Q), nq, _p(ex), k, _p(ids), _p(d))
    return ids, d


def knn_graph_rows(X: np.ndarray, rows, R: int):
    """Rows of the exact kNN graph: for each listed i, the R nearest j != i."""
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    return knn(X, X[rows], R, exclude=rows)


def splitmix64(seed: int, count: int) -> np.ndarray:
    out = np.empty(count, np.uint64)
    lib().orc_splitmix64(C.c_uint64(seed), count, _p(out))
    return out


def init_rows(n: int, K: int, seed: int) -> np.ndarray:
    out = np.empty(K, np.int64)
    lib().orc_init_rows(n, K, C.c_uint64(seed), _p(out))
    return out


def kmeans(X: np.ndarray, P: int, K: int, iters: int, seed: int, want_assign: bool = False):
    """Per-subspace k-means codebooks, shape (P, K, d/P), dtype of X."""
    X = np.ascontiguousarray(X)
    n, d = X.shape
    cb = np.empty((P, K, d // P), X.dtype)
    asg = np.empty((n, P), np.int32) if want_assign else None
    lib().orc_kmeans(_p(X), n, d, _dt(X), P, K, iters, C.c_uint64(seed), _p(cb), _p(asg))
    return (cb, asg) if want_assign else cb


def tables(q: np.ndarray, codebooks: np.ndarray) -> np.ndarray:
    """(P, K) squared distances from each query subvector to its codewords."""
    P, K, ds = codebooks.shape
    q = np.ascontiguousarray(q, dtype=codebooks.dtype)
    cb = np.ascontiguousarray(codebooks)
    tab = np.empty((P, K), np.float64)
    lib().orc_tables(_p(q), P * ds, _dt(cb), P, K, _p(cb), _p(tab))
    return tab


def sort_tables(tab: np.ndarray):
    """Each row ascending by (value, index): returns (perm int32, sorted float64)."""
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    P, K = tab.shape
    perm = np.empty((P, K), np.int32)
    srt = np.empty((P, K), np.float64)
    lib().orc_sort_tables(P, K, _p(tab), _p(perm), _p(srt))
    return perm, srt


def mseq(tab: np.ndarray, count: int):
    """First `count` bridges in increasing distance: (lids int64, sums, max heap size)."""
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    P, K = tab.shape
    lids = np.empty(count, np.int64)
    sums = np.empty(count, np.float64)
    mh = np.zeros(1, np.int64)
    got = lib().orc_mseq(P, K, _p(tab), count, _p(lids), _p(sums), _p(mh))
    return lids[:got], sums[:got], int(mh[0])


def bridge_graph(X: np.ndarray, codebooks: np.ndarray, t: int, b: int):
    """Bridge graph as CSR: (off uint32[K^P+1], ids uint32[E], dist float64[E])."""
    X = np.ascontiguousarray(X)
    n, d = X.shape
    P, K, _ = codebooks.shape
    nb = K ** P
    tt = min(t, nb)
    cap = n * tt if b <= 0 else min(n * tt, b * nb)
    off = np.empty(nb + 1, np.uint32)
    ids = np.empty(max(cap, 1), np.uint32)
    bd = np.empty(max(cap, 1), np.float64)
    e = lib().orc_bridge_graph(_p(X), n, d, _dt(X), P, K, _p(np.ascontiguousarray(codebooks)), t, b,
                               _p(off), _p(ids), _p(bd), cap)
    if e < 0:
        raise RuntimeError("bridge graph capacity exceeded")
    return off, ids[:e].copy(), bd[:e].copy()


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Nearest bfloat16 value of each float32 (ties to an even last bit), as float64."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty(x.shape, np.float64)
    lib().orc_bf16_round(_p(x), x.size, _p(out))
    return out


def search(X, codebooks, graph, off, ids, Q, k, T, L, trace_len: int = 0, stats: bool = False,
           precision: int = 0, rerank_k: int = 0, seeds=None):
    """Alg. 1 on the given index.  k and T may be scalars or per-query arrays.
    precision 1 (float data): bfloat16 rows drive the search, the best
    max(k, rerank_k) are re-ranked on the float rows.  seeds (array of ids):
    the graph search without bridges, the seeds measured first.
    Returns (ids int32 nq x kmax, dists float64 nq x kmax[, trace][, stats])."""
    X = np.ascontiguousarray(X)
    n, d = X.shape
    P, K, _ = codebooks.shape
    Q = np.ascontiguousarray(Q, dtype=X.dtype)
    nq = Q.shape[0]
    ks = np.broadcast_to(np.asarray(k, np.int32), (nq,)).copy()
    Ts = np.broadcast_to(np.asarray(T, np.int32), (nq,)).copy()
    kmax = int(ks.max()) if nq else 1
    graph = np.ascontiguousarray(graph, dtype=np.uint32)
    R = graph.shape[1] if graph.ndim == 2 else 0
    if graph.size == 0:
        graph = np.zeros(1, np.uint32)
    off = np.ascontiguousarray(off, dtype=np.uint32)
    ids_ = np.ascontiguousarray(ids, dtype=np.uint32)
    if ids_.size == 0:
        ids_ = np.zeros(1, np.uint32)
    oid = np.empty((nq, kmax), np.int32)
    od = np.empty((nq, kmax), np.float64)
    tr = np.empty((nq, trace_len), np.int32) if trace_len > 0 else None
    st = np.empty((nq, 6), np.int64) if stats else None
    sd = None if seeds is None else np.ascontiguousarray(seeds, dtype=np.uint32)
    lib().orc_search_ex(_p(X), n, d, _dt(X), P, K, _p(np.ascontiguousarray(codebooks)), R, _p(graph), _p(off),
                        _p(ids_), _p(Q), nq, _p(ks), _p(Ts), kmax, L, precision, rerank_k, 1 if sd is None else 0,
                        _p(sd), 0 if sd is None else len(sd), _p(oid), _p(od), _p(tr), trace_len, _p(st))
    out = [oid, od]
    if tr is not None:
        out.append(tr)
    if st is not None:
        out.append(st)
    return tuple(out)


def build_index(X: np.ndarray, P: int, K: int, R: int, iters: int, seed: int, t: int, b: int):
    """The whole index the oracle's way: codebooks, exact kNN graph, bridge CSR."""
    cb = kmeans(X, P, K, iters, seed)
    n = X.shape[0]
    g, _ = knn_graph_rows(X, np.arange(n), R) if R > 0 else (np.zeros((n, 0), np.int32), None)
    off, ids, _ = bridge_graph(X, cb, t, b)
    return cb, g.astype(np.uint32), off, ids


def pq_encode(R: np.ndarray, codebooks: np.ndarray, want_gap: bool = False):
    """Residual codes (Sec. 5): per subspace the nearest codeword of
    codebooks (m, K, d/m) float32, ties to the smaller index.  R (n, d) is
    taken in double precision.  With want_gap also the second-best minus the
    best squared distance per code."""
    R = np.ascontiguousarray(R, np.float64)
    cb = np.ascontiguousarray(codebooks, np.float32)
    n, d = R.shape
    m, K, _ = cb.shape
    codes = np.empty((n, m), np.uint8)
    gap = np.empty((n, m), np.float64) if want_gap else None
    lib().orc_pq_encode(_p(R), n, d, m, K, _p(cb), _p(codes), _p(gap))
    return (codes, gap) if want_gap else codes


def ivf_adc(Q: np.ndarray, centres: np.ndarray, list_off: np.ndarray, list_ids: np.ndarray, codes: np.ndarray,
            codebooks: np.ndarray, lists: np.ndarray, L: int, k: int, want_count: bool = False):
    """Graph-D-ADC re-ranking (Sec. 5): each query's lists (nq, W) in
    visiting order (-1 skipped), candidates cut at exactly L, ranked by
    |q - c - r|^2 then id.  Returns (ids (nq, k) int32, dists (nq, k))."""
    Q = np.ascontiguousarray(Q, np.uint8)
    centres = np.ascontiguousarray(centres, np.uint8)
    list_off = np.ascontiguousarray(list_off, np.uint32)
    list_ids = np.ascontiguousarray(list_ids, np.uint32)
    codes = np.ascontiguousarray(codes, np.uint8)
    cb = np.ascontiguousarray(codebooks, np.float32)
    lists = np.ascontiguousarray(lists, np.int32)
    nq, d = Q.shape
    m, K, _ = cb.shape
    W = lists.shape[1]
    ids = np.empty((nq, k), np.int32)
    dd = np.empty((nq, k), np.float64)
    cnt = np.empty(nq, np.int64)
    lib().orc_ivf_adc(_p(Q), nq, d, _p(centres), _p(list_off), _p(list_ids), _p(codes), m, K, _p(cb), _p(lists),
                      W, int(L), k, _p(ids), _p(dd), _p(cnt))
    return (ids, dd, cnt) if want_count else (ids, dd)
