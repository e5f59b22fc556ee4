"""Independent, deliberately naive re-derivations used to pin the oracle.

Nothing here calls the oracle or the GPU library.  These are brute-force or
restated forms of the paper's definitions, valid only for tiny inputs:

* ``brute_knn``: linear scan (Sec. 1, Sec. 5.1 ground truth) with numpy,
  ties by id via lexsort.
* ``all_bridges``: every one of the K^P concatenated bridge vectors written
  out explicitly (Sec. 4.1, Cartesian concatenation), with its distance to
  the query computed on the full vector, not from tables.
* ``literal_search``: the evaluation order of Alg. 1 (Sec. 4.2) stated as a
  merge of two ordered streams.  Bridge vectors are consumed in the order of
  an explicit sort of ``all_bridges``; reference vectors come from a
  best-first frontier kept as a sorted list and cut back to its L best
  after every insertion (L = None: no cut).  The next vertex expanded is
  whichever stream's head is smaller in (distance, node id).  Holding every
  bridge in the sorted stream expands the same vertices in the same order
  as extracting one bridge at a time, because a bridge never precedes the
  one before it.  Strict budget; (distance, node id) ties.
* ``seeded_graph_search``: the neighborhood-graph search of Sec. 2.2 with no
  bridge graph: fixed seed vectors are measured first, then the frontier is
  expanded best first.
"""
from __future__ import annotations

import bisect
import itertools

import numpy as np


def sqdist(a, b) -> float:
    if np.asarray(a).dtype == np.uint8:
        diff = np.asarray(a, np.int64) - np.asarray(b, np.int64)
        return float(np.sum(diff * diff))
    diff = np.asarray(a, np.float64) - np.asarray(b, np.float64)
    return float(np.sum(diff * diff))


def brute_knn(X, Q, k, exclude=None):
    """ids (nq, k), dists (nq, k) ascending by (D, id); padded with -1 / inf."""
    if X.dtype == np.uint8:
        Xi = X.astype(np.int64)
        Qi = Q.astype(np.int64)
    else:
        Xi = X.astype(np.float64)
        Qi = Q.astype(np.float64)
    ids = np.full((len(Q), k), -1, np.int64)
    ds = np.full((len(Q), k), np.inf)
    for i, q in enumerate(Qi):
        D = ((Xi - q) ** 2).sum(axis=1).astype(np.float64)
        idx = np.arange(len(X))
        if exclude is not None and exclude[i] >= 0:
            keep = idx != exclude[i]
            D, idx = D[keep], idx[keep]
        order = np.lexsort((idx, D))[:k]
        ids[i, : len(order)] = idx[order]
        ds[i, : len(order)] = D[order]
    return ids, ds


def all_bridges(codebooks):
    """Every bridge vector y_lid, lid = sum_p k_p K^(P-1-p): array (K^P, d)."""
    P, K, ds = codebooks.shape
    ys = []
    for tup in itertools.product(range(K), repeat=P):  # row-major: subspace 0 most significant
        ys.append(np.concatenate([codebooks[p, tup[p]] for p in range(P)]))
    return np.stack(ys)


def bridge_order(q, codebooks):
    """(lid, distance) of every bridge, sorted by (distance, lid)."""
    ys = all_bridges(codebooks)
    D = np.array([sqdist(q, y) for y in ys])
    order = np.lexsort((np.arange(len(ys)), D))
    return [(int(l), float(D[l])) for l in order]


def _expand_stream(X, graph, q, T, L, head_lists, bridge_stream, bridge_lists):
    """Shared walk of the two streams.  head_lists: lists of ids measured
    before anything else (the seeds of a graph search), in order."""
    n = len(X)
    seen = set()
    trace, measured = [], []
    frontier = []          # sorted (distance, id), at most L long
    bi = 0

    def visit(ids):
        for x in ids:
            if len(trace) == T:
                return
            x = int(x)
            if x in seen:
                continue
            seen.add(x)
            key = (sqdist(q, X[x]), x)
            trace.append(x)
            measured.append(key)
            bisect.insort(frontier, key)
            if L is not None and len(frontier) > L:
                frontier.pop()           # the worst entry leaves (possibly the new one)

    for ids in head_lists:
        visit(ids)
    while len(trace) < T:
        nb = bridge_stream[bi] if bi < len(bridge_stream) else None
        nf = frontier[0] if frontier else None
        if nb is None and nf is None:
            break
        if nf is None or (nb is not None and (nb[1], n + nb[0]) < nf):
            bi += 1
            visit(bridge_lists.get(nb[0], []))
        else:
            frontier.pop(0)
            visit(graph[nf[1]])
    return trace, measured


def _topk(measured, k):
    best = sorted(measured)[:k]
    ids = [x for _, x in best] + [-1] * max(0, k - len(best))
    ds = [d for d, _ in best] + [np.inf] * max(0, k - len(best))
    return ids, ds


def literal_search(X, codebooks, graph, bridge_lists, q, k, T, L=None):
    """Alg. 1 as a merge of the sorted bridge stream and a best-first frontier
    of at most L references.  bridge_lists: dict lid -> list of reference ids.
    Returns (trace, ids, dists)."""
    trace, measured = _expand_stream(X, graph, q, T, L, [], bridge_order(q, codebooks), bridge_lists)
    ids, ds = _topk(measured, k)
    return trace, ids, ds


def seeded_graph_search(X, graph, seeds, q, k, T, L=None):
    """Neighborhood-graph search without bridges (Sec. 2.2): the seeds are
    measured in the given order, then the frontier is expanded best first."""
    trace, measured = _expand_stream(X, graph, q, T, L, [seeds], [], {})
    ids, ds = _topk(measured, k)
    return trace, ids, ds


def bf16_round(x):
    """float32 -> nearest bfloat16 value (ties to an even last bit), as float64.
    Written from the definition: bfloat16 keeps the top 16 bits of the float32
    pattern; the two candidates are the patterns just below and just above."""
    x = np.asarray(x, np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lo = (u & 0xFFFF0000).astype(np.uint32).view(np.float32).astype(np.float64)
    hi_bits = ((u & 0xFFFF0000) + 0x10000).astype(np.uint32)
    hi = hi_bits.view(np.float32).astype(np.float64)
    xv = x.astype(np.float64)
    dlo, dhi = np.abs(xv - lo), np.abs(hi - xv)
    lo_even = ((u >> 16) & 1) == 0
    pick_lo = (dlo < dhi) | ((dlo == dhi) & lo_even)
    return np.where(pick_lo, lo, hi)


def csr_to_lists(off, ids):
    return {lid: [int(v) for v in ids[off[lid]:off[lid + 1]]]
            for lid in range(len(off) - 1) if off[lid + 1] > off[lid]}


def parse_golden(path):
    """Parse tests/golden/toy_2d_search.txt."""
    cbs, pts, graph, bridges, queries = {}, [], {}, {}, []
    with open(path) as f:
        for raw in f:
            line = raw.split("#", 1)[0].strip()
            if not line or line == "points:":
                continue
            if line.startswith("codebook"):
                head, vals = line.split(":")
                cbs[int(head.split()[1])] = [int(v) for v in vals.split()]
            elif line.startswith("graph"):
                head, vals = line.split(":")
                graph[int(head.split()[1][1:])] = [int(v) for v in vals.split()]
            elif line.startswith("bridge"):
                head, vals = line.split(":")
                bridges[int(head.split()[1][1:])] = [int(v) for v in vals.split()]
            elif line.startswith("query"):
                queries.append({"q": [int(v) for v in line.split()[1:]], "cases": []})
            elif line.startswith("case"):
                parts = [p.strip() for p in line[4:].split("|")]
                k, T, L = (int(v) for v in parts[0].split())
                trace = [int(v) for v in parts[1].split()]
                ids = [int(v) for v in parts[2].split()]
                ds = [float(v) for v in parts[3].split()]
                queries[-1]["cases"].append(dict(k=k, T=T, L=L, trace=trace, ids=ids, dists=ds))
            elif line.startswith("x"):
                v = line.split()
                pts.append([int(a) for a in v[1:]])
    P = len(cbs)
    K = len(cbs[0])
    codebooks = np.array([[[c] for c in cbs[p]] for p in range(P)], np.uint8)
    X = np.array(pts, np.uint8)
    G = np.array([graph[i] for i in range(len(pts))], np.uint32)
    return dict(codebooks=codebooks, X=X, graph=G, bridges=bridges, queries=queries, K=K, P=P)
