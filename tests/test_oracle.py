"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test states what fixes the expected value: a published test vector, a
hand-traced example, a closed form, a brute-force re-derivation on tiny
inputs, or an invariant of the method (Sec. 3.3, Sec. 4.1, Sec. 4.2, Alg. 1).
"""
import os

import numpy as np
import pytest

import oracle
from tests import literal

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "toy_2d_search.txt")


def tiny_u8(rng, n, d, hi=256):
    return rng.integers(0, hi, size=(n, d)).astype(np.uint8)


def tiny_index(rng, n=60, d=8, P=2, K=4, R=4, hi=8, t=1, b=0, iters=3, seed=7):
    X = tiny_u8(rng, n, d, hi)
    cb = oracle.kmeans(X, P, K, iters, seed)
    g, _ = oracle.knn_graph_rows(X, np.arange(n), R)
    off, ids, _ = oracle.bridge_graph(X, cb, t, b)
    return X, cb, g.astype(np.uint32), off, ids


# ---------------------------------------------------------------- generators

def test_splitmix64_published_vectors():
    # SplitMix64 reference outputs (Steele, Lea, Flood 2014 / Vigna's reference code):
    # seed 0 and seed 1234567 (the latter also used by Java's SplittableRandom tests).
    got0 = [int(v) for v in oracle.splitmix64(0, 4)]
    assert got0 == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    got1 = [int(v) for v in oracle.splitmix64(1234567, 3)]
    assert got1 == [6457827717110365317, 3203168211198807973, 9817491932198370423]


def test_init_rows_partial_permutation():
    rows = oracle.init_rows(1000, 64, 99)
    assert len(set(rows.tolist())) == 64 and rows.min() >= 0 and rows.max() < 1000
    full = oracle.init_rows(50, 50, 5)
    assert sorted(full.tolist()) == list(range(50))
    # the first draw picks index (x mod n) of the identity permutation
    first = int(oracle.splitmix64(123, 1)[0] % np.uint64(777))
    assert oracle.init_rows(777, 1, 123)[0] == first


# ---------------------------------------------------------------- brute force (V1)

@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_knn_matches_numpy_bruteforce(dtype):
    rng = np.random.default_rng(3)
    if dtype == "u8":
        X = tiny_u8(rng, 300, 16, hi=4)    # many exact ties
        Q = tiny_u8(rng, 20, 16, hi=4)
    else:
        X = rng.standard_normal((300, 12)).astype(np.float32)
        Q = rng.standard_normal((20, 12)).astype(np.float32)
    for k in (1, 7, 300, 305):
        ids, ds = oracle.knn(X, Q, k)
        eids, eds = literal.brute_knn(X, Q, k)
        np.testing.assert_array_equal(ids, eids)
        if dtype == "u8":
            np.testing.assert_array_equal(ds, eds)
        else:  # summation order differs from numpy's pairwise sum
            np.testing.assert_allclose(ds, eds, rtol=1e-12)


def test_knn_graph_excludes_self_and_is_sorted():
    rng = np.random.default_rng(4)
    X = tiny_u8(rng, 200, 8, hi=3)
    X[5] = X[6]  # duplicate vectors stay neighbours at distance 0
    rows = np.arange(200)
    g, gd = oracle.knn_graph_rows(X, rows, 6)
    eg, egd = literal.brute_knn(X, X, 6, exclude=rows)
    np.testing.assert_array_equal(g, eg)
    np.testing.assert_array_equal(gd, egd)
    assert (g != rows[:, None]).all()
    assert g[5, 0] == 6 and gd[5, 0] == 0


# ---------------------------------------------------------------- hand-traced example

def test_golden_graph_and_bridge_graph():
    gd = literal.parse_golden(GOLDEN)
    X, cb = gd["X"], gd["codebooks"]
    g, _ = oracle.knn_graph_rows(X, np.arange(len(X)), 2)
    np.testing.assert_array_equal(g, gd["graph"])
    off, ids, _ = oracle.bridge_graph(X, cb, 1, 0)
    assert literal.csr_to_lists(off, ids) == gd["bridges"]


def test_golden_search_cases():
    gd = literal.parse_golden(GOLDEN)
    X, cb, G = gd["X"], gd["codebooks"], gd["graph"]
    off = np.zeros(gd["K"] ** gd["P"] + 1, np.uint32)
    flat = []
    for lid in range(gd["K"] ** gd["P"]):
        off[lid] = len(flat)
        flat += gd["bridges"].get(lid, [])
    off[-1] = len(flat)
    ids = np.array(flat, np.uint32)
    ncase = 0
    for qd in gd["queries"]:
        q = np.array([qd["q"]], np.uint8)
        for c in qd["cases"]:
            T = c["T"]
            rid, rdist, tr = oracle.search(X, cb, G, off, ids, q, c["k"], T, c["L"], trace_len=max(T, 1))
            assert rid[0].tolist() == c["ids"], c
            assert rdist[0].tolist() == c["dists"], c
            assert [v for v in tr[0].tolist() if v >= 0] == c["trace"], c
            # the two-stream form reproduces the same hand trace
            ltr, lid_, ld = literal.literal_search(X, cb, G, gd["bridges"], q[0], c["k"], T, L=c["L"])
            assert ltr == c["trace"] and lid_ == c["ids"] and ld == c["dists"]
            ncase += 1
    assert ncase == 8


# ---------------------------------------------------------------- tables (V4)

@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_tables_sum_to_full_bridge_distance(dtype):
    rng = np.random.default_rng(5)
    P, K, ds = 3, 4, 4
    if dtype == "u8":
        cb = rng.integers(0, 256, size=(P, K, ds)).astype(np.uint8)
        q = rng.integers(0, 256, size=P * ds).astype(np.uint8)
    else:
        cb = rng.standard_normal((P, K, ds)).astype(np.float32)
        q = rng.standard_normal(P * ds).astype(np.float32)
    tab = oracle.tables(q, cb)
    ys = literal.all_bridges(cb)
    for lid, y in enumerate(ys):
        ks = np.unravel_index(lid, (K,) * P)
        s = sum(tab[p, ks[p]] for p in range(P))
        full = literal.sqdist(q, y)
        if dtype == "u8":
            assert s == full
        else:
            assert abs(s - full) <= 1e-12 * max(1.0, full)


def test_sort_tables_order_and_ties():
    tab = np.array([[3, 1, 3, 0, 1], [2, 2, 2, 2, 2]], np.float64)
    perm, srt = oracle.sort_tables(tab)
    assert perm[0].tolist() == [3, 1, 4, 0, 2]
    assert perm[1].tolist() == [0, 1, 2, 3, 4]
    assert srt[0].tolist() == [0, 1, 1, 3, 3]


# ---------------------------------------------------------------- multi-sequence (V3, V8)

@pytest.mark.parametrize("P,K", [(1, 7), (2, 5), (3, 4), (4, 3), (2, 16)])
def test_mseq_equals_sort_of_all_tuples(P, K):
    rng = np.random.default_rng(100 * P + K)
    for trial in range(40):
        hi = 3 if trial % 2 == 0 else 1000      # tie-heavy and tie-free tables
        tab = rng.integers(0, hi, size=(P, K)).astype(np.float64)
        total = K ** P
        lids, sums, maxheap = oracle.mseq(tab, total + 5)
        assert len(lids) == total
        allsum = np.zeros(total)
        for lid in range(total):
            ks = np.unravel_index(lid, (K,) * P)
            allsum[lid] = sum(tab[p, ks[p]] for p in range(P))
        order = np.lexsort((np.arange(total), allsum))
        np.testing.assert_array_equal(lids, order)
        np.testing.assert_array_equal(sums, allsum[order])
        # the heap grows by at most P-1 per extraction (one pop, at most P pushes)
        assert maxheap <= 1 + (P - 1) * total
        # a prefix request gives the prefix
        l5, s5, _ = oracle.mseq(tab, 5)
        np.testing.assert_array_equal(l5, order[:5])


def test_mseq_P1_is_sorted_table():
    tab = np.array([[5.0, 2.0, 2.0, 9.0, 0.0]])
    lids, sums, mh = oracle.mseq(tab, 10)
    assert lids.tolist() == [4, 1, 2, 0, 3]
    assert sums.tolist() == [0.0, 2.0, 2.0, 5.0, 9.0]
    assert mh == 1


def test_mseq_matches_full_vector_bridge_order():
    rng = np.random.default_rng(8)
    cb = rng.integers(0, 6, size=(3, 3, 2)).astype(np.uint8)
    q = rng.integers(0, 6, size=6).astype(np.uint8)
    lids, sums, _ = oracle.mseq(oracle.tables(q, cb), 27)
    ref = literal.bridge_order(q, cb)
    assert [(int(a), float(b)) for a, b in zip(lids, sums)] == ref


# ---------------------------------------------------------------- bridge graph (V10)

def test_bridge_graph_nearest_bridge_rule():
    rng = np.random.default_rng(9)
    X = tiny_u8(rng, 400, 8, hi=16)
    P, K = 2, 4
    cb = oracle.kmeans(X, P, K, 4, 11)
    off, ids, bd = oracle.bridge_graph(X, cb, 1, 0)
    assert off[-1] == len(X) and sorted(ids.tolist()) == list(range(len(X)))
    ys = literal.all_bridges(cb)
    for lid in range(K ** P):
        lst = ids[off[lid]:off[lid + 1]]
        dd = bd[off[lid]:off[lid + 1]]
        keys = list(zip(dd.tolist(), lst.tolist()))
        assert keys == sorted(keys)
        for i, dv in zip(lst, dd):
            D = np.array([literal.sqdist(X[i], y) for y in ys])
            best = int(np.lexsort((np.arange(len(ys)), D))[0])
            assert best == lid and D[best] == dv


@pytest.mark.parametrize("t,b", [(3, 0), (3, 2), (5, 1), (100, 0)])
def test_bridge_graph_top_t_top_b_bruteforce(t, b):
    rng = np.random.default_rng(10 + t + b)
    X = tiny_u8(rng, 120, 6, hi=5)
    cb = rng.integers(0, 5, size=(3, 3, 2)).astype(np.uint8)
    off, ids, bd = oracle.bridge_graph(X, cb, t, b)
    ys = literal.all_bridges(cb)
    nb = len(ys)
    tt = min(t, nb)
    lists = {lid: [] for lid in range(nb)}
    for i in range(len(X)):
        D = np.array([literal.sqdist(X[i], y) for y in ys])
        for lid in np.lexsort((np.arange(nb), D))[:tt]:
            lists[int(lid)].append((D[lid], i))
    for lid in range(nb):
        exp = sorted(lists[lid])
        if b > 0:
            exp = exp[:b]
        got = list(zip(bd[off[lid]:off[lid + 1]].tolist(), ids[off[lid]:off[lid + 1]].tolist()))
        assert got == exp


# ---------------------------------------------------------------- k-means (V12)

def test_kmeans_replay_last_update():
    rng = np.random.default_rng(12)
    X = tiny_u8(rng, 500, 12)
    P, K = 3, 6
    cb, asg = oracle.kmeans(X, P, K, 5, 77, want_assign=True)
    assert cb.dtype == np.uint8
    ds = 12 // P
    prev = oracle.kmeans(X, P, K, 4, 77)   # centroids the last assignment was made against
    for p in range(P):
        sub = X[:, p * ds:(p + 1) * ds].astype(np.int64)
        # the recorded assignment is the nearest previous centroid, ties to the smaller index
        D = ((sub[:, None, :] - prev[p][None, :, :].astype(np.int64)) ** 2).sum(-1)
        np.testing.assert_array_equal(asg[:, p], D.argmin(axis=1))
        for j in range(K):
            m = asg[:, p] == j
            if not m.any():
                np.testing.assert_array_equal(cb[p, j], prev[p, j])
                continue
            s = sub[m].sum(0)
            n = int(m.sum())
            # mean rounded half up, in exact integers
            exp = np.floor(s / n + 0.5).astype(np.int64)
            np.testing.assert_array_equal(cb[p, j].astype(np.int64), exp)


def test_kmeans_zero_iters_are_init_rows():
    rng = np.random.default_rng(13)
    X = tiny_u8(rng, 300, 8)
    cb = oracle.kmeans(X, 2, 5, 0, 42)
    rows = oracle.init_rows(300, 5, 42)
    np.testing.assert_array_equal(cb[0], X[rows, :4])
    np.testing.assert_array_equal(cb[1], X[rows, 4:])


def test_kmeans_single_cluster_is_rounded_mean():
    X = np.array([[0, 10], [1, 11], [2, 11], [3, 13]], np.uint8)
    cb = oracle.kmeans(X, 1, 1, 3, 1)
    # means 1.5 -> 2 (half up), 11.25 -> 11
    assert cb[0, 0].tolist() == [2, 11]


def test_kmeans_separated_clusters_f32():
    rng = np.random.default_rng(14)
    centres = np.array([[0.0, 0.0], [100.0, 0.0], [0.0, 100.0]])
    X = np.concatenate([c + rng.standard_normal((50, 2)) for c in centres]).astype(np.float32)
    # take the first seed whose initial rows land in three different clusters
    seed = next(s for s in range(1000) if len(set((oracle.init_rows(150, 3, s) // 50).tolist())) == 3)
    cb = oracle.kmeans(X, 1, 3, 10, seed)
    got = sorted(map(tuple, cb[0].astype(np.float64).round(6)))
    exp = sorted(tuple(X[i * 50:(i + 1) * 50].astype(np.float64).mean(0).round(6)) for i in range(3))
    np.testing.assert_allclose(got, exp, rtol=0, atol=1e-5)


# ---------------------------------------------------------------- whole search

def test_exhaustive_budget_returns_exact_knn():
    """V2: every reference linked to a bridge and T >= N, so the search sees all of X."""
    rng = np.random.default_rng(15)
    for trial in range(6):
        X, cb, g, off, ids = tiny_index(rng, n=80, d=8, P=2, K=3, R=3, hi=6 if trial % 2 else 256)
        Q = tiny_u8(rng, 10, 8, hi=6 if trial % 2 else 256)
        for k in (1, 10, 80):
            rid, rd = oracle.search(X, cb, g, off, ids, Q, k, len(X), 16)
            eid, ed = literal.brute_knn(X, Q, k)
            np.testing.assert_array_equal(rid, eid)
            np.testing.assert_array_equal(rd, ed)


@pytest.mark.parametrize("trial", range(8))
def test_search_matches_literal_single_queue(trial):
    """V9: with L >= T the bounded queue plus bridge slot equals the paper's single queue."""
    rng = np.random.default_rng(200 + trial)
    P = 1 + trial % 3
    X, cb, g, off, ids = tiny_index(rng, n=70, d=6 if P == 3 else 8, P=P, K=3, R=3, hi=4 + 60 * (trial % 2),
                                    t=1 + (trial % 2), b=(trial % 3))
    lists = literal.csr_to_lists(off, ids)
    Q = tiny_u8(rng, 6, X.shape[1], hi=4 + 60 * (trial % 2))
    for T in (1, 7, 25, 70):
        rid, rd, tr = oracle.search(X, cb, g, off, ids, Q, 5, T, T, trace_len=T)
        for i in range(len(Q)):
            ltr, lid_, ld = literal.literal_search(X, cb, g, lists, Q[i], 5, T)
            assert [v for v in tr[i].tolist() if v >= 0] == ltr
            assert rid[i].tolist() == lid_
            assert rd[i].tolist() == ld


@pytest.mark.parametrize("trial", range(10))
def test_bounded_queue_matches_literal_eviction(trial):
    """Reading 5 with L < T: a frontier cut back to its L best after each
    insertion (the two-stream form) expands the same vertices in the same
    order as the oracle's bounded queue with worst-eviction, on tie-heavy
    and tie-free data, with every bridge rule."""
    rng = np.random.default_rng(500 + trial)
    P = 1 + trial % 3
    hi = 4 if trial % 2 == 0 else 256
    X, cb, g, off, ids = tiny_index(rng, n=90, d=6 if P == 3 else 8, P=P, K=3, R=4, hi=hi,
                                    t=1 + (trial % 3), b=(trial % 4))
    lists = literal.csr_to_lists(off, ids)
    Q = tiny_u8(rng, 5, X.shape[1], hi=hi)
    for L in (1, 2, 5, 17):
        for T in (9, 40, 90):
            rid, rd, tr = oracle.search(X, cb, g, off, ids, Q, 6, T, L, trace_len=T)
            for i in range(len(Q)):
                ltr, lid_, ld = literal.literal_search(X, cb, g, lists, Q[i], 6, T, L=L)
                assert [v for v in tr[i].tolist() if v >= 0] == ltr, (L, T, i)
                assert rid[i].tolist() == lid_
                assert rd[i].tolist() == ld


def test_bounded_queue_differs_from_unbounded():
    """The bound is not vacuous: on these inputs a queue of L = 1 expands
    other vertices than the unbounded queue (both forms agree on which)."""
    rng = np.random.default_rng(42)
    X, cb, g, off, ids = tiny_index(rng, n=120, d=8, P=2, K=3, R=4, hi=256, t=1, b=0)
    lists = literal.csr_to_lists(off, ids)
    Q = tiny_u8(rng, 6, 8)
    differ = 0
    for i in range(len(Q)):
        a, _, _ = literal.literal_search(X, cb, g, lists, Q[i], 5, 60, L=1)
        b, _, _ = literal.literal_search(X, cb, g, lists, Q[i], 5, 60)
        differ += a != b
    assert differ > 0


def test_search_f32_matches_literal():
    rng = np.random.default_rng(31)
    X = rng.standard_normal((90, 8)).astype(np.float32)
    cb = oracle.kmeans(X, 2, 3, 4, 5)
    g, _ = oracle.knn_graph_rows(X, np.arange(90), 4)
    off, ids, _ = oracle.bridge_graph(X, cb, 2, 3)
    lists = literal.csr_to_lists(off, ids)
    Q = rng.standard_normal((5, 8)).astype(np.float32)
    rid, rd, tr = oracle.search(X, cb, g, off, ids, Q, 4, 30, 30, trace_len=30)
    for i in range(5):
        ltr, lid_, ld = literal.literal_search(X, cb, g, lists, Q[i], 4, 30)
        assert [v for v in tr[i].tolist() if v >= 0] == ltr
        assert rid[i].tolist() == lid_
        np.testing.assert_allclose(rd[i], ld, rtol=1e-12)


def test_budget_prefix_property():
    """V5: the evaluation sequence does not depend on T or k."""
    rng = np.random.default_rng(16)
    X, cb, g, off, ids = tiny_index(rng, n=300, d=8, P=2, K=4, R=5, hi=256, t=2, b=3)
    Q = tiny_u8(rng, 8, 8)
    _, _, long_tr = oracle.search(X, cb, g, off, ids, Q, 10, 200, 8, trace_len=200)
    for T in (1, 13, 64, 150):
        _, _, tr = oracle.search(X, cb, g, off, ids, Q, 10, T, 8, trace_len=T)
        np.testing.assert_array_equal(tr, long_tr[:, :T])
    i100, d100 = oracle.search(X, cb, g, off, ids, Q, 100, 150, 8)
    i10, d10 = oracle.search(X, cb, g, off, ids, Q, 10, 150, 8)
    np.testing.assert_array_equal(i100[:, :10], i10)
    np.testing.assert_array_equal(d100[:, :10], d10)


def test_graph_free_search_is_inverted_multi_index_order():
    """V7: with no kNN edges, t=1 and all references kept, the references come out
    ordered by (rank of their bridge, distance to that bridge, id)."""
    rng = np.random.default_rng(17)
    X = tiny_u8(rng, 150, 8, hi=20)
    cb = oracle.kmeans(X, 2, 4, 3, 3)
    off, ids, bd = oracle.bridge_graph(X, cb, 1, 0)
    g = np.zeros((150, 0), np.uint32)
    Q = tiny_u8(rng, 4, 8, hi=20)
    _, _, tr = oracle.search(X, cb, g, off, ids, Q, 10, 150, 64, trace_len=150)
    ys = literal.all_bridges(cb)
    own = np.empty(150, np.int64)
    dist_own = np.empty(150)
    for i in range(150):
        D = np.array([literal.sqdist(X[i], y) for y in ys])
        own[i] = np.lexsort((np.arange(len(ys)), D))[0]
        dist_own[i] = D[own[i]]
    for qi in range(4):
        rank = {lid: r for r, (lid, _) in enumerate(literal.bridge_order(Q[qi], cb))}
        order = sorted(range(150), key=lambda i: (rank[int(own[i])], dist_own[i], i))
        assert tr[qi].tolist() == order


def test_bounded_queue_changes_only_through_eviction():
    """A tiny L still evaluates exactly T vectors while work remains, and the result
    equals the top-k of the vectors it evaluated."""
    rng = np.random.default_rng(18)
    X, cb, g, off, ids = tiny_index(rng, n=200, d=8, P=2, K=4, R=4, t=1, b=0)
    Q = tiny_u8(rng, 6, 8)
    rid, rd, tr = oracle.search(X, cb, g, off, ids, Q, 5, 60, 1, trace_len=60)
    for i in range(6):
        ev = [v for v in tr[i] if v >= 0]
        assert len(ev) == 60 and len(set(ev)) == 60
        D = [literal.sqdist(Q[i], X[v]) for v in ev]
        best = sorted(zip(D, ev))[:5]
        assert rid[i].tolist() == [v for _, v in best]


def test_degenerate_inputs():
    rng = np.random.default_rng(19)
    X, cb, g, off, ids = tiny_index(rng, n=30, d=8, P=2, K=3, R=3)
    Q = tiny_u8(rng, 3, 8)
    rid, rd = oracle.search(X, cb, g, off, ids, Q, 4, 0, 64)
    assert (rid == -1).all() and np.isinf(rd).all()
    rid, rd = oracle.search(X, cb, g, off, ids, Q, 40, 1000, 64)
    assert (rid[:, 30:] == -1).all() and (rid[:, :30] >= 0).all()
    # a single reference vector
    X1 = np.array([[7, 9]], np.uint8)
    cb1 = oracle.kmeans(X1, 1, 1, 2, 0)
    off1, ids1, _ = oracle.bridge_graph(X1, cb1, 1, 0)
    rid, rd = oracle.search(X1, cb1, np.zeros((1, 0), np.uint32), off1, ids1,
                            np.array([[0, 0]], np.uint8), 2, 5, 4)
    assert rid.tolist() == [[0, -1]] and rd[0, 0] == 130.0


# ---------------------------------------------------------------- bf16 precision form

def test_bf16_rounding_matches_library_conversion():
    """The oracle's bfloat16 rounding against torch's float32 -> bfloat16
    conversion (round to nearest even), including exact halfway cases."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(40)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        np.abs(rng.standard_normal(5000))]).astype(np.float32)
    # halfway between two bfloat16 values: low 16 bits exactly 0x8000
    half = (rng.integers(0x3F000000, 0x41000000, 4000, dtype=np.uint64) & ~np.uint64(0xFFFF)) | np.uint64(0x8000)
    x = np.concatenate([x, half.astype(np.uint32).view(np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(oracle.bf16_round(x), ref)
    np.testing.assert_array_equal(literal.bf16_round(x), ref)


def _f32_index(rng, n=120, d=8, P=2, K=3, R=4, t=2, b=3):
    X = rng.standard_normal((n, d)).astype(np.float32)
    cb = oracle.kmeans(X, P, K, 3, 5)
    g, _ = oracle.knn_graph_rows(X, np.arange(n), R)
    off, ids, _ = oracle.bridge_graph(X, cb, t, b)
    return X, cb, g.astype(np.uint32), off, ids


@pytest.mark.parametrize("rerank_k", [0, 3, 12])
def test_bf16_search_is_exact_search_on_rounded_rows_then_rerank(rerank_k):
    """Precision form: the traversal equals the two-stream search run on the
    bfloat16-rounded rows (float query), and the answer is the best
    max(k, rerank_k) of what it measured, measured again on the float rows."""
    rng = np.random.default_rng(41 + rerank_k)
    X, cb, g, off, ids = _f32_index(rng)
    lists = literal.csr_to_lists(off, ids)
    Q = rng.standard_normal((6, 8)).astype(np.float32)
    Xb = literal.bf16_round(X)
    k = 4
    for L, T in ((64, 50), (3, 80)):
        rid, rd, tr = oracle.search(X, cb, g, off, ids, Q, k, T, L, trace_len=T, precision=1, rerank_k=rerank_k)
        for i in range(len(Q)):
            ltr, _, _ = literal.literal_search(Xb, cb, g, lists, Q[i], k, T, L=L)
            assert [v for v in tr[i].tolist() if v >= 0] == ltr
            approx = sorted((literal.sqdist(Q[i], Xb[x]), x) for x in ltr)[:max(k, rerank_k)]
            exact = sorted((literal.sqdist(Q[i], X[x]), x) for _, x in approx)[:k]
            assert rid[i].tolist() == [x for _, x in exact]
            np.testing.assert_allclose(rd[i], [dd for dd, _ in exact], rtol=1e-12)


def test_bf16_search_on_representable_rows_equals_exact_search():
    """Rows whose values are bfloat16 numbers already: both precisions agree."""
    rng = np.random.default_rng(43)
    X = rng.integers(-50, 50, size=(100, 8)).astype(np.float32) / 4
    cb = oracle.kmeans(X, 2, 3, 3, 5)
    g, _ = oracle.knn_graph_rows(X, np.arange(100), 4)
    off, ids, _ = oracle.bridge_graph(X, cb, 2, 3)
    Q = rng.standard_normal((5, 8)).astype(np.float32)
    a = oracle.search(X, cb, g.astype(np.uint32), off, ids, Q, 5, 60, 8, trace_len=60)
    b = oracle.search(X, cb, g.astype(np.uint32), off, ids, Q, 5, 60, 8, trace_len=60, precision=1)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)


# ---------------------------------------------------------------- graph search without bridges (Sec. 2.2)

@pytest.mark.parametrize("trial", range(6))
def test_seeded_graph_search_matches_literal(trial):
    rng = np.random.default_rng(600 + trial)
    hi = 4 if trial % 2 == 0 else 256
    X, cb, g, off, ids = tiny_index(rng, n=100, d=8, P=2, K=3, R=3 + trial % 3, hi=hi)
    Q = tiny_u8(rng, 5, 8, hi=hi)
    seeds = rng.choice(100, size=1 + trial * 2, replace=False).astype(np.uint32)
    if trial == 3:
        seeds = np.concatenate([seeds, seeds[:2]])        # repeated seeds are measured once
    for L, T in ((64, 70), (2, 40), (7, 100)):
        rid, rd, tr = oracle.search(X, cb, g, off, ids, Q, 5, T, L, trace_len=T, seeds=seeds)
        for i in range(len(Q)):
            ltr, lid_, ld = literal.seeded_graph_search(X, g, seeds, Q[i], 5, T, L=L)
            assert [v for v in tr[i].tolist() if v >= 0] == ltr
            assert rid[i].tolist() == lid_ and rd[i].tolist() == ld


def test_seeded_graph_search_closed_forms():
    rng = np.random.default_rng(44)
    X, cb, g, off, ids = tiny_index(rng, n=80, d=8, P=2, K=3, R=3, hi=256)
    Q = tiny_u8(rng, 4, 8)
    # no graph edges: exactly the seeds, in order, up to the budget
    seeds = np.array([5, 9, 2, 77, 40], np.uint32)
    _, _, tr = oracle.search(X, cb, np.zeros((80, 0), np.uint32), off, ids, Q, 3, 4, 64, trace_len=4, seeds=seeds)
    assert (tr == seeds[:4]).all()
    # every vector a seed and T >= n: the exact nearest neighbours
    allseeds = rng.permutation(80).astype(np.uint32)
    rid, rd = oracle.search(X, cb, g, off, ids, Q, 10, 80, 64, seeds=allseeds)
    eid, ed = literal.brute_knn(X, Q, 10)
    np.testing.assert_array_equal(rid, eid)
    np.testing.assert_array_equal(rd, ed)


# ---------------------------------------------------------------- Graph-D-ADC (Sec. 5)

def _adc_example():
    """Worked by hand.  d = 4, two subspaces of two codewords each.
    List 0 (centre 10,10,10,10): ids 2 (code 1,0) and 5 (code 0,1);
    list 1 (centre 0,0,0,0): id 7 (code 1,1); list 2 (centre 5,5,5,5): ids 9
    and 4, both code 0,0.  Query 11,12,9,10:
      id 2: q - c - r = (0, 0, -1, 0)        -> 1
      id 5: q - c - r = (1, 2, 2, -0.5)      -> 9.25
      id 7: q - c - r = (10, 10, 12, 9.5)    -> 434.25
      ids 9 and 4: q - c = (6, 7, 4, 5)      -> 126 (a tie: 4 before 9)"""
    centres = np.array([[10, 10, 10, 10], [0, 0, 0, 0], [5, 5, 5, 5]], np.uint8)
    cb = np.array([[[0, 0], [1, 2]], [[0, 0], [-3, 0.5]]], np.float32)
    list_off = np.array([0, 2, 3, 5], np.uint32)
    list_ids = np.array([2, 5, 7, 9, 4], np.uint32)
    codes = np.array([[1, 0], [0, 1], [1, 1], [0, 0], [0, 0]], np.uint8)
    q = np.array([[11, 12, 9, 10]], np.uint8)
    return q, centres, list_off, list_ids, codes, cb


@pytest.mark.parametrize("order,L,k,ids,dists,count", [
    ([0, 1, 2], 5, 5, [2, 5, 4, 9, 7], [1, 9.25, 126, 126, 434.25], 5),
    ([1, 0], 2, 3, [2, 7, -1], [1, 434.25, np.inf], 2),          # list 0 cut after its first vector
    ([2, -1, 0], 3, 3, [2, 4, 9], [1, 126, 126], 3),             # -1 skipped, cut inside list 0
    ([0, 1, 2], 0, 2, [-1, -1], [np.inf, np.inf], 0),
    ([0, 1, 2], 100, 2, [2, 5], [1, 9.25], 5),
])
def test_ivf_adc_hand_example(order, L, k, ids, dists, count):
    q, centres, off, lids, codes, cb = _adc_example()
    got, gd, cnt = oracle.ivf_adc(q, centres, off, lids, codes, cb, np.array([order]), L, k, want_count=True)
    assert got[0].tolist() == ids
    np.testing.assert_array_equal(gd[0], np.array(dists, np.float64))
    assert cnt[0] == count


def test_pq_encode_matches_bruteforce_argmin():
    """Nearest codeword per subspace, first index on ties (numpy's argmin),
    with duplicated codewords planted so that ties occur."""
    rng = np.random.default_rng(11)
    n, d, m, K = 50, 8, 4, 16
    R = rng.integers(-6, 7, size=(n, d)).astype(np.float64)
    cb = rng.integers(-6, 7, size=(m, K, d // m)).astype(np.float32)
    cb[0, 9] = cb[0, 3]
    cb[2, 15] = cb[2, 0]
    R[:5, 0:2] = cb[0, 3]                 # exactly on the duplicated codeword
    codes, gap = oracle.pq_encode(R, cb, want_gap=True)
    ds = d // m
    for p in range(m):
        D = ((R[:, None, p * ds:(p + 1) * ds] - cb[p][None].astype(np.float64)) ** 2).sum(-1)
        np.testing.assert_array_equal(codes[:, p], D.argmin(1))
        S = np.sort(D, 1)
        np.testing.assert_array_equal(gap[:, p], S[:, 1] - S[:, 0])
    assert (codes[:5, 0] == 3).all() and (gap[:5, 0] == 0).all()


@pytest.mark.parametrize("L", [10_000, 37])
def test_ivf_adc_with_exact_codes_is_exact_knn(L):
    """Codebooks holding every residual subvector reproduce each vector
    exactly, so with every list visited and no cut the re-ranking is the
    brute-force k-nearest-neighbour list by (distance, id); with a cut it is
    the brute-force list over the first L vectors in list order."""
    rng = np.random.default_rng(12)
    n, d, m, K, C, k = 60, 8, 2, 64, 3, 10
    X = rng.integers(0, 12, size=(n, d)).astype(np.uint8)
    centres = X[[4, 17, 33]]
    Dc = ((X[:, None, :].astype(np.int64) - centres[None].astype(np.int64)) ** 2).sum(-1)
    assign = Dc.argmin(1)
    R = X.astype(np.float64) - centres[assign].astype(np.float64)
    ds = d // m
    cb = rng.integers(-12, 13, size=(m, K, ds)).astype(np.float32)
    for p in range(m):
        slots = rng.permutation(K)[:n]
        cb[p, slots] = R[:, p * ds:(p + 1) * ds]
    codes_v = oracle.pq_encode(R, cb)
    for p in range(m):
        np.testing.assert_array_equal(cb[p, codes_v[:, p]].astype(np.float64), R[:, p * ds:(p + 1) * ds])
    list_ids = np.concatenate([np.flatnonzero(assign == j) for j in range(C)]).astype(np.uint32)
    list_off = np.concatenate([[0], np.cumsum(np.bincount(assign, minlength=C))]).astype(np.uint32)
    codes = codes_v[list_ids]
    Q = rng.integers(0, 12, size=(7, d)).astype(np.uint8)
    order = np.tile(np.array([[2, 0, 1]], np.int32), (len(Q), 1))
    ids, dd = oracle.ivf_adc(Q, centres, list_off, list_ids, codes, cb, order, L, k)
    pool = np.concatenate([list_ids[list_off[j]:list_off[j + 1]] for j in (2, 0, 1)])[:L].astype(np.int64)
    for qi in range(len(Q)):
        exact = ((X[pool].astype(np.int64) - Q[qi].astype(np.int64)) ** 2).sum(1)
        o = np.lexsort((pool, exact))[:k]
        np.testing.assert_array_equal(ids[qi], pool[o])
        np.testing.assert_array_equal(dd[qi], exact[o].astype(np.float64))
