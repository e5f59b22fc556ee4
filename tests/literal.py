"""Independent, deliberately naive re-derivations used to pin the oracle.

Nothing here calls the oracle or the GPU library.  These are brute-force or
literal forms of the paper's definitions, valid only for tiny inputs:

* ``brute_knn``: linear scan (Sec. 1, Sec. 5.1 ground truth) with numpy,
  ties by id via lexsort.
* ``all_bridges``: every one of the K^P concatenated bridge vectors written
  out explicitly (Sec. 4.1, Cartesian concatenation), with its distance to
  the query computed on the full vector, not from tables.
* ``literal_search``: Alg. 1 with ONE unbounded main queue that holds
  reference and bridge vectors together (Sec. 4.2: "the main queue consists
  of only one bridge vector if available"), the bridge order taken from the
  explicit sort of ``all_bridges``.  Strict budget, (distance, node id) ties.
"""
from __future__ import annotations

import heapq
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


def literal_search(X, codebooks, graph, bridge_lists, q, k, T):
    """Alg. 1 with one unbounded priority queue over references and bridges.
    bridge_lists: dict lid -> list of reference ids.  Returns (trace, ids, dists)."""
    n = len(X)
    border = bridge_order(q, codebooks)
    nxt = iter(border)
    color = np.zeros(n, bool)
    Qh = []
    b = next(nxt, None)
    if b is not None:
        heapq.heappush(Qh, (b[1], n + b[0]))
    t, trace, res = 0, [], []
    while Qh and t < T:
        D, node = heapq.heappop(Qh)
        if node >= n:
            adj = bridge_lists.get(node - n, [])
        else:
            adj = list(graph[node])
        for x in adj:
            if t == T:
                break
            x = int(x)
            if color[x]:
                continue
            color[x] = True
            dx = sqdist(q, X[x])
            heapq.heappush(Qh, (dx, x))
            res.append((dx, x))
            trace.append(x)
            t += 1
        if node >= n:
            b = next(nxt, None)
            if b is not None:
                heapq.heappush(Qh, (b[1], n + b[0]))
    res.sort()
    ids = [x for _, x in res[:k]] + [-1] * max(0, k - len(res))
    ds = [d for d, _ in res[:k]] + [np.inf] * max(0, k - len(res))
    return trace, ids, ds


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
