"""GPU vs oracle parity through the C ABI.

u8 results must be bit-exact: codebooks, kNN graph, bridge CSR, returned ids,
int32 distances and the evaluation order.  Sizes are chosen so that the
oracle finishes in seconds while the kernels still run many tiles, chunks
and ragged tails.
"""
import numpy as np
import pytest

import oracle
from paper_1312_3062_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _index_cls():
    from paper_1312_3062_amd import Index
    return Index


def gpu_search(idx, Q, k, T, L=64, ks=None, Ts=None, trace=False, stats=False, precision=0, rerank_k=0):
    qd = torch.from_numpy(np.ascontiguousarray(Q)).cuda()
    nq = Q.shape[0]
    tr = torch.empty((nq, max(T, 1)), dtype=torch.int32, device="cuda") if trace else None
    st = torch.empty((nq, 12), dtype=torch.int32, device="cuda") if stats else None
    kd = None if ks is None else torch.from_numpy(np.asarray(ks, np.int32)).cuda()
    td = None if Ts is None else torch.from_numpy(np.asarray(Ts, np.int32)).cuda()
    ids, dd = _index_cls().search_device(idx, qd, k, T, ks=kd, budgets=td, queue_len=L, trace=tr, stats=st,
                                         precision=precision, rerank_k=rerank_k)
    torch.cuda.synchronize()
    out = [ids.cpu().numpy(), dd.cpu().numpy()]
    if trace:
        out.append(tr.cpu().numpy())
    if stats:
        out.append(st.cpu().numpy())
    return out


def assert_search_equal(idx, parts, X, Q, k, T, L, **kw):
    gi, gd, gt = gpu_search(idx, Q, k, T, L, trace=True, **kw)
    ks = kw.get("ks", k)
    Ts = kw.get("Ts", T)
    oi, od, ot = oracle.search(X, parts["codebooks"], parts["graph"], parts["bridge_off"], parts["bridge_ids"], Q,
                               ks, Ts, L, trace_len=max(T, 1))
    np.testing.assert_array_equal(gi, oi)
    np.testing.assert_array_equal(gd.astype(np.float64), np.where(np.isinf(od), 2147483647.0, od))
    if T > 0:
        np.testing.assert_array_equal(gt, ot)


# ---------------------------------------------------------------- the 10K x 128 u8 workload, in full

@pytest.fixture(scope="module")
def tiny():
    w = synth.WORKLOADS["tiny_10k_u8"]
    X = synth.base_vectors(w)
    Q = synth.queries(w)
    idx = _index_cls().build(X, w.graph_k, w.P, w.K, w.kmeans_iters, w.kmeans_seed, w.bridge_t, w.bridge_b)
    parts = idx.export()
    return dict(w=w, X=X, Q=Q, idx=idx, parts=parts)


@pytest.fixture(scope="module")
def tiny_oracle(tiny):
    w, X = tiny["w"], tiny["X"]
    cb = oracle.kmeans(X, w.P, w.K, w.kmeans_iters, w.kmeans_seed)
    g, _ = oracle.knn_graph_rows(X, np.arange(len(X)), w.graph_k)
    off, ids, _ = oracle.bridge_graph(X, cb, w.bridge_t, w.bridge_b)
    return dict(codebooks=cb, graph=g.astype(np.uint32), bridge_off=off, bridge_ids=ids)


def test_tiny_codebooks_bit_exact(tiny, tiny_oracle):
    np.testing.assert_array_equal(tiny["parts"]["codebooks"], tiny_oracle["codebooks"])


def test_tiny_knn_graph_bit_exact(tiny, tiny_oracle):
    np.testing.assert_array_equal(tiny["parts"]["graph"], tiny_oracle["graph"])


def test_tiny_bridge_csr_bit_exact(tiny, tiny_oracle):
    np.testing.assert_array_equal(tiny["parts"]["bridge_off"], tiny_oracle["bridge_off"])
    np.testing.assert_array_equal(tiny["parts"]["bridge_ids"], tiny_oracle["bridge_ids"])


def test_tiny_search_bit_exact(tiny):
    w = tiny["w"]
    assert_search_equal(tiny["idx"], tiny["parts"], tiny["X"], tiny["Q"], w.k, 256, w.queue_len)


@pytest.mark.parametrize("k,T,L", [(1, 0, 64), (10, 1, 64), (10, 17, 1), (100, 300, 7), (5, 1000, 64),
                                   (33, 129, 2), (1, 64, 64)])
def test_tiny_search_budget_grid(tiny, k, T, L):
    Q = tiny["Q"][:40]
    assert_search_equal(tiny["idx"], tiny["parts"], tiny["X"], Q, k, T, L)


def test_tiny_per_query_k_and_budget(tiny):
    rng = np.random.default_rng(0)
    Q = tiny["Q"]
    ks = rng.choice([1, 10, 100], size=len(Q)).astype(np.int32)
    Ts = rng.integers(0, 700, size=len(Q)).astype(np.int32)
    assert_search_equal(tiny["idx"], tiny["parts"], tiny["X"], Q, 100, 700, 64, ks=ks, Ts=Ts)


def test_tiny_stats_are_consistent(tiny):
    Q = tiny["Q"]
    gi, gd, st = gpu_search(tiny["idx"], Q, 10, 256, 64, stats=True)
    assert (st[:, 0] <= 256).all() and (st[:, 6] == 0).all()
    _, _, _, ost = oracle.search(tiny["X"], tiny["parts"]["codebooks"], tiny["parts"]["graph"],
                                 tiny["parts"]["bridge_off"], tiny["parts"]["bridge_ids"], Q, 10, 256, 64,
                                 trace_len=1, stats=True)
    np.testing.assert_array_equal(st[:, 0], ost[:, 0])   # evaluations
    np.testing.assert_array_equal(st[:, 1], ost[:, 1])   # reference pops


def test_tiny_tables_bit_exact(tiny):
    Q = tiny["Q"][:20]
    sv, perm = tiny["idx"].tables_device(torch.from_numpy(Q).cuda())
    torch.cuda.synchronize()
    sv, perm = sv.cpu().numpy(), perm.cpu().numpy()
    for i in range(len(Q)):
        tab = oracle.tables(Q[i], tiny["parts"]["codebooks"])
        op, osv = oracle.sort_tables(tab)
        np.testing.assert_array_equal(perm[i], op)
        np.testing.assert_array_equal(sv[i].astype(np.float64), osv)


def test_knn_device_matches_oracle(tiny):
    from paper_1312_3062_amd import knn_device
    X, Q = tiny["X"], tiny["Q"]
    xd = torch.from_numpy(X).cuda()
    qd = torch.from_numpy(Q).cuda()
    for k in (1, 10, 32):
        ids, dd = knn_device(xd, qd, k)
        torch.cuda.synchronize()
        oi, od = oracle.knn(X, Q, k)
        np.testing.assert_array_equal(ids.cpu().numpy(), oi)
        np.testing.assert_array_equal(dd.cpu().numpy().astype(np.float64), od)


@pytest.mark.parametrize("n,nq,d,k,dups", [
    (1000, 37, 128, 10, 0),     # matrix cores: ragged tile and query block
    (4163, 300, 64, 32, 40),    # duplicated rows: ties broken by id
    (777, 1, 192, 1, 5),
    (2050, 257, 256, 16, 0),
    (530, 70, 48, 7, 3),        # VALU path (d not a multiple of 64)
])
def test_knn_device_shapes_and_ties(n, nq, d, k, dups):
    from paper_1312_3062_amd import knn_device
    rng = np.random.default_rng(n + d)
    X = rng.integers(0, 256, size=(n, d)).astype(np.uint8)
    if dups:
        X[rng.choice(n, dups, replace=False)] = X[rng.choice(n, dups)]
    Q = np.concatenate([X[:nq // 2], rng.integers(0, 256, size=(nq - nq // 2, d)).astype(np.uint8)])
    xd = torch.from_numpy(X).cuda()
    ids, dd = knn_device(xd, torch.from_numpy(Q).cuda(), k)
    torch.cuda.synchronize()
    oi, od = oracle.knn(X, Q, k)
    np.testing.assert_array_equal(ids.cpu().numpy(), oi)
    np.testing.assert_array_equal(dd.cpu().numpy().astype(np.float64), od)
    # the graph form: each row's k nearest others
    gi, gd = knn_device(xd, xd, k, exclude_self=True)
    torch.cuda.synchronize()
    rows = np.arange(0, n, max(1, n // 97))
    oi, od = oracle.knn_graph_rows(X, rows, k)
    np.testing.assert_array_equal(gi.cpu().numpy()[rows], oi)
    np.testing.assert_array_equal(gd.cpu().numpy()[rows].astype(np.float64), od)


@pytest.mark.parametrize("n,nq,d,k", [(3000, 70, 384, 10), (2100, 300, 128, 32), (900, 5, 256, 1), (700, 40, 96, 16)])
def test_knn_device_f32_within_tolerance(n, nq, d, k):
    """fp32 kNN (matrix cores for d in {128, 256, 384}) against the fp64 oracle:
    returned distances within 1e-5 relative, ids equal except where fp32
    rounding reorders a near tie."""
    from paper_1312_3062_amd import knn_device
    rng = np.random.default_rng(d + k)
    X = np.abs(rng.standard_normal((n, d))).astype(np.float32)
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    Q = np.abs(rng.standard_normal((nq, d))).astype(np.float32)
    Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    xd = torch.from_numpy(X).cuda()
    for q, excl in ((Q, False), (X, True)):
        ids, dd = knn_device(xd, torch.from_numpy(q).cuda(), k, exclude_self=excl)
        torch.cuda.synchronize()
        ids, dd = ids.cpu().numpy(), dd.cpu().numpy().astype(np.float64)
        oi, od = oracle.knn(X, q, k, exclude=np.arange(len(q)) if excl else None)
        np.testing.assert_allclose(dd, od, rtol=1e-5)
        ex = ((X[ids].astype(np.float64) - q.astype(np.float64)[:, None, :]) ** 2).sum(2)
        np.testing.assert_allclose(dd, ex, rtol=1e-5)
        assert (ids == oi).mean() >= 0.99


def test_import_and_save_load_roundtrip(tiny, tiny_oracle, tmp_path):
    Index = _index_cls()
    X = tiny["X"]
    imp = Index.from_parts(X, tiny_oracle["codebooks"], tiny_oracle["graph"], tiny_oracle["bridge_off"],
                           tiny_oracle["bridge_ids"])
    assert_search_equal(imp, tiny_oracle, X, tiny["Q"], 10, 256, 64)
    path = str(tmp_path / "tiny.annidx")
    imp.save(path)
    back = Index.load(path)
    p2 = back.export()
    for key in ("codebooks", "graph", "bridge_off", "bridge_ids"):
        np.testing.assert_array_equal(p2[key], tiny_oracle[key])
    gi, gd = gpu_search(back, tiny["Q"], 10, 256, 64)
    hi, hd = back.search(tiny["Q"], 10, 256, 64)
    np.testing.assert_array_equal(gi, hi)
    np.testing.assert_array_equal(gd, hd)


def test_exhaustive_budget_returns_exact_knn():
    """t=1, all references kept, T >= n: the search reaches every vector."""
    w = synth.scaled(synth.WORKLOADS["tiny_10k_u8"], 1500, nq=30, K=8)
    X, Q = synth.base_vectors(w), synth.queries(w)
    idx = _index_cls().build(X, 6, 2, 8, 5, 9, 1, 0)
    gi, gd = gpu_search(idx, Q, 20, 1500, 64)
    oi, od = oracle.knn(X, Q, 20)
    np.testing.assert_array_equal(gi, oi)
    np.testing.assert_array_equal(gd.astype(np.float64), od)


# ---------------------------------------------------------------- small variants, full build parity

VARIANTS = [
    # n, d, P, K, R, t, b, iters, hi
    (700, 16, 1, 9, 5, 1, 0, 3, 256),
    (900, 32, 2, 5, 8, 3, 2, 4, 6),      # tie-heavy values
    (1000, 48, 3, 4, 7, 5, 0, 2, 256),
    (1200, 64, 4, 6, 12, 100, 5, 3, 256),
    (800, 128, 4, 3, 3, 2, 1, 1, 4),     # tie-heavy, tiny lists
    (1300, 256, 2, 16, 16, 4, 3, 6, 256),
    (600, 512, 4, 8, 6, 2, 0, 2, 256),   # the largest u8 rows (512 bytes) and distances
]


@pytest.mark.parametrize("n,d,P,K,R,t,b,iters,hi", VARIANTS)
def test_variant_build_and_search_bit_exact(n, d, P, K, R, t, b, iters, hi):
    rng = np.random.default_rng(n + d + P)
    X = rng.integers(0, hi, size=(n, d)).astype(np.uint8)
    X[7] = X[3]                               # duplicate vectors
    Q = rng.integers(0, hi, size=(25, d)).astype(np.uint8)
    Q[0] = X[5]                               # a query equal to a reference vector
    idx = _index_cls().build(X, R, P, K, iters, 1234, t, b)
    parts = idx.export()
    cb = oracle.kmeans(X, P, K, iters, 1234)
    np.testing.assert_array_equal(parts["codebooks"], cb)
    g, _ = oracle.knn_graph_rows(X, np.arange(n), R)
    np.testing.assert_array_equal(parts["graph"], g)
    off, ids, _ = oracle.bridge_graph(X, cb, t, b)
    np.testing.assert_array_equal(parts["bridge_off"], off)
    np.testing.assert_array_equal(parts["bridge_ids"], ids)
    for k, T, L in ((10, 200, 64), (3, 57, 1), (50, n, 16)):
        assert_search_equal(idx, parts, X, Q, k, T, L)


@pytest.mark.parametrize("n,d,P,K,hi", [
    (3000, 192, 2, 256, 256),   # 96-byte subvectors (a partial second k-slice), the most codewords
    (2500, 80, 1, 200, 8),      # 80 bytes, a partial last block of codewords, tie-heavy values
])
def test_kmeans_on_matrix_cores_bit_exact(n, d, P, K, hi):
    """The u8 k-means assignment on matrix cores: codebooks bit-exact against
    the oracle's k-means (ties to the smaller codeword)."""
    rng = np.random.default_rng(n + K)
    X = rng.integers(0, hi, size=(n, d)).astype(np.uint8)
    idx = _index_cls().build(X, 4, P, K, 3, 99, 1, 0)
    np.testing.assert_array_equal(idx.export()["codebooks"], oracle.kmeans(X, P, K, 3, 99))


def test_graph_free_index():
    """R = 0: only bridge lists are expanded."""
    rng = np.random.default_rng(5)
    X = rng.integers(0, 256, size=(600, 32)).astype(np.uint8)
    Q = rng.integers(0, 256, size=(10, 32)).astype(np.uint8)
    idx = _index_cls().build(X, 0, 2, 6, 3, 7, 1, 0)
    parts = idx.export()
    assert_search_equal(idx, parts, X, Q, 10, 600, 64)


# ---------------------------------------------------------------- f32: tolerance against the FP64 oracle

def test_f32_search_within_tolerance():
    w = synth.scaled(synth.WORKLOADS["gist_like_1m_f32"], 4000, nq=50, K=12, d=96, P=3)
    X, Q = synth.base_vectors(w), synth.queries(w)
    idx = _index_cls().build(X, 8, 3, 12, 5, 3, 4, 3)
    parts = idx.export()
    gi, gd = gpu_search(idx, Q, 10, 300, 64)
    oi, od = oracle.search(X, parts["codebooks"], parts["graph"], parts["bridge_off"], parts["bridge_ids"], Q,
                           10, 300, 64)
    # distances of the returned ids, recomputed in fp64, against the GPU's fp32 values
    for i in range(len(Q)):
        ex = ((X[gi[i]].astype(np.float64) - Q[i].astype(np.float64)) ** 2).sum(1)
        np.testing.assert_allclose(gd[i], ex, rtol=1e-4)
    gt, _ = oracle.knn(X, Q, 10)
    from paper_1312_3062_amd import recall_at
    assert abs(recall_at(gi, gt, 10) - recall_at(oi, gt, 10)) <= 0.002 + 1e-12
    # bf16 gather with fp32 re-rank: returned distances are fp32-exact for the returned ids
    bi, bd = gpu_search(idx, Q, 10, 300, 64, precision=1, rerank_k=20)
    for i in range(len(Q)):
        ex = ((X[bi[i]].astype(np.float64) - Q[i].astype(np.float64)) ** 2).sum(1)
        np.testing.assert_allclose(bd[i], ex, rtol=1e-4)
        assert (np.diff(bd[i]) >= 0).all()


# ---------------------------------------------------------------- bridge-heavy searches

@pytest.mark.parametrize("n,P,K,t,b,T,k", [
    (3000, 4, 8, 10, 5, 2000, 10),    # short lists fetched ahead with their distances
    (2500, 3, 12, 6, 3, 2400, 20),    # P = 3: one side of two lists, one of one
    (2000, 2, 40, 4, 2, 1900, 5),     # P = 2: both sides plain lists
    (4000, 4, 9, 25, 0, 3900, 10),    # all kept: long lists walked from memory
])
def test_bridge_heavy_search_bit_exact(n, P, K, t, b, T, k):
    rng = np.random.default_rng(n + K)
    X = rng.integers(0, 256, size=(n, 48)).astype(np.uint8)
    Q = rng.integers(0, 256, size=(20, 48)).astype(np.uint8)
    # a sparse graph (R = 2) exhausts its neighbourhoods quickly; bridges take over
    idx = _index_cls().build(X, 2, P, K, 3, 99, t, b)
    parts = idx.export()
    gi, gd, st = gpu_search(idx, Q, k, T, 64, stats=True)
    assert (st[:, 2] > 40).all()            # many bridges expanded per query
    assert (st[:, 6] == 0).all()
    assert_search_equal(idx, parts, X, Q, k, T, 64)


def test_state_capacity_by_batch_size():
    """Three lists of 100 codewords: a batch that stays resident with 512
    multi-sequence elements per query in LDS gets them, a larger batch gets
    256 (short bridge lists are fetched ahead either way).  Both give the
    oracle's results, query by query."""
    rng = np.random.default_rng(31)
    n = 6000
    X = rng.integers(0, 256, size=(n, 48)).astype(np.uint8)
    Q = rng.integers(0, 256, size=(3000, 48)).astype(np.uint8)
    idx = _index_cls().build(X, 8, 3, 100, 3, 17, 10, 5)
    parts = idx.export()
    gi, gd, st = gpu_search(idx, Q, 10, 600, 64, stats=True)        # more than the chip holds at 512
    si, sd = gpu_search(idx, Q[:200], 10, 600, 64)                  # resident at 512
    assert (st[:, 6] == 0).all()
    assert (st[:, 2] > 5).mean() > 0.5       # bridges are expanded throughout
    np.testing.assert_array_equal(si, gi[:200])
    np.testing.assert_array_equal(sd, gd[:200])
    rows = np.arange(0, len(Q), 5)          # every fifth query against the oracle
    oi, od = oracle.search(X, parts["codebooks"], parts["graph"], parts["bridge_off"], parts["bridge_ids"], Q[rows],
                           10, 600, 64)
    np.testing.assert_array_equal(gi[rows], oi)
    np.testing.assert_array_equal(gd[rows].astype(np.float64), np.where(np.isinf(od), 2147483647.0, od))


def _overflow_case(dtype=np.uint8):
    """65,536 bridges with lists of one.  The fp32 case holds integers and
    keeps the sampled codewords (no k-means iteration), so that every fp32
    distance, table entry and sum is an exact integer: the float kernels then
    match the oracle bit for bit, like the u8 ones."""
    rng = np.random.default_rng(77)
    n = 2000
    X = rng.integers(0, 256, size=(n, 32)).astype(dtype)
    Q = rng.integers(0, 256, size=(12, 32)).astype(dtype)
    iters = 2 if dtype == np.uint8 else 0
    idx = _index_cls().build(X, 1, 4, 16, iters, 5, 3, 1)
    return X, Q, idx, idx.export()


@pytest.mark.parametrize("dtype", [np.uint8, np.float32], ids=["u8", "f32"])
def test_multisequence_overflow_moves_to_a_global_slot_exactly(dtype):
    """At T <= 2048, with four lists of at most 64 codewords, the LDS
    enumeration holds 8 elements per side; a query that needs more carries on
    with its state in a global slot."""
    X, Q, idx, parts = _overflow_case(dtype)
    gi, gd, st = gpu_search(idx, Q, 10, 1800, 64, stats=True)
    assert (st[:, 10] == 1).any()           # some queries outgrew the LDS capacity
    assert (st[:, 9] == 0).all()            # ... and found a free slot
    assert (st[:, 6] == 0).all()
    assert_search_equal(idx, parts, X, Q, 10, 1800, 64)


@pytest.mark.parametrize("dtype", [np.uint8, np.float32], ids=["u8", "f32"])
def test_multisequence_overflow_without_a_free_slot_is_rerun_exactly(dtype):
    """A workspace with room for one global slot: queries that find it taken
    are searched again by the second kernel, with the same results."""
    X, Q, idx, parts = _overflow_case(dtype)
    nq, k, T = len(Q), 10, 1800
    # at this budget the full workspace has one slot of several KB per query
    # (12 <= 256) and a few hundred bytes of lists: 3/(2 nq) of it holds the
    # lists and one slot, not two
    small = torch.empty(idx.workspace_bytes(nq, k, T) * 3 // (2 * nq), dtype=torch.uint8, device="cuda")
    qd = torch.from_numpy(Q).cuda()
    st = torch.empty((nq, 12), dtype=torch.int32, device="cuda")
    ids, dd = idx.search_device(qd, k, T, stats=st, workspace=small)
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    assert ((st[:, 9] == 1) | (st[:, 10] == 1)).sum() >= 2
    assert (st[:, 9] == 1).any()            # the slot was in use: re-run
    assert (st[:, 6] == 0).all()
    oi, od = oracle.search(X, parts["codebooks"], parts["graph"], parts["bridge_off"], parts["bridge_ids"], Q,
                           k, T, 64)
    np.testing.assert_array_equal(ids.cpu().numpy(), oi)
    np.testing.assert_array_equal(dd.cpu().numpy().astype(np.float64), np.where(np.isinf(od), 2147483647.0, od))


# ---------------------------------------------------------------- edge cases

@pytest.mark.parametrize("k,T", [(129, 700), (500, 900), (1024, 1500)])
def test_large_k_bit_exact(tiny, k, T):
    """Result sets beyond 128 keys (16 per lane), up to the 1024 maximum."""
    Q = tiny["Q"][:12]
    assert_search_equal(tiny["idx"], tiny["parts"], tiny["X"], Q, k, T, 64)


def test_empty_batch_and_zero_budget(tiny):
    idx = tiny["idx"]
    qd = torch.empty((0, tiny["X"].shape[1]), dtype=torch.uint8, device="cuda")
    ids, dd = idx.search_device(qd, 10, 256)
    torch.cuda.synchronize()
    assert ids.shape == (0, 10) and dd.shape == (0, 10)
    gi, gd = gpu_search(idx, tiny["Q"][:5], 7, 0, 64)
    assert (gi == -1).all() and (gd == 2147483647).all()


# ---------------------------------------------------------------- bf16 gather against the oracle's bf16 form

@pytest.mark.parametrize("rerank_k", [0, 20])
def test_bf16_search_against_the_oracle_bf16_form(rerank_k):
    """The bf16 traversal (bf16 rows, fp32 query and accumulation) against the
    oracle's bf16 form (the same rows, rounded to nearest even, in fp64),
    then the fp32 re-rank: ids equal on this small GIST-shaped index, returned
    distances within 1e-4 relative of fp64 and of the oracle's."""
    w = synth.scaled(synth.WORKLOADS["gist_like_1m_f32"], 4000, nq=60, K=12, d=96, P=3)
    X, Q = synth.base_vectors(w), synth.queries(w)
    idx = _index_cls().build(X, 8, 3, 12, 5, 3, 4, 3)
    p = idx.export()
    ks = np.random.default_rng(rerank_k).choice([1, 10, 25], size=len(Q)).astype(np.int32)
    for T, L in ((300, 64), (900, 5)):
        gi, gd = gpu_search(idx, Q, 25, T, L, ks=ks, precision=1, rerank_k=rerank_k)
        oi, od = oracle.search(X, p["codebooks"], p["graph"], p["bridge_off"], p["bridge_ids"], Q, ks, T, L,
                               precision=1, rerank_k=rerank_k)
        np.testing.assert_array_equal(gi, oi)
        fin = oi >= 0
        np.testing.assert_allclose(gd[fin], od[fin], rtol=1e-4)
        assert np.isinf(gd[~fin]).all()


# ---------------------------------------------------------------- fp32 build against the oracle

def test_f32_build_against_the_oracle():
    """fp32 index build on a small GIST-shaped set.
    Codebooks: the GPU sums members in int64 fixed point (order-free, far
    finer than an fp32 ulp here) and divides in fp32; the oracle sums and
    divides in fp64.  A centroid element then differs by a few fp32 ulps
    (rtol 1e-5, atol 1e-6 on values of order 0.05), provided no assignment
    flips on a near tie.  A fp32 distance over ds dims is within ds * 2^-24
    relative of the exact one (ds products and ds sums, each rounded once);
    the test checks that the nearest and second-nearest centroid of every
    point differ by more than twice that for both distances, 4 ds 2^-24,
    in every iteration.
    Tables: fp32 subspace sums against fp64 within 1e-5 relative, and the
    same codeword at every rank separated from its neighbours by more.
    Bridge lists (built from the oracle's codebooks): equal to the oracle's
    lists, except that a list may differ where fp32 rounding reorders
    distances that agree to 1e-5 (each such list is checked against fp64
    distances with that tolerance, and at most 1% of lists may differ)."""
    from tests import literal
    w = synth.scaled(synth.WORKLOADS["gist_like_1m_f32"], 3000, nq=40, K=10, d=96, P=3)
    X, Q = synth.base_vectors(w), synth.queries(w)
    P, K, ds, iters, seed, t, b = 3, 10, 32, 6, 11, 3, 4
    idx = _index_cls().build(X, 6, P, K, iters, seed, t, b)
    p = idx.export()
    cb = oracle.kmeans(X, P, K, iters, seed)
    for it in range(iters):
        prev = oracle.kmeans(X, P, K, it, seed)      # the centroids iteration `it` assigns against
        for s in range(P):
            sub = X[:, s * ds:(s + 1) * ds].astype(np.float64)
            D = ((sub[:, None, :] - prev[s][None].astype(np.float64)) ** 2).sum(-1)
            D.sort(axis=1)
            assert ((D[:, 1] - D[:, 0]) / D[:, 1]).min() > 4 * ds * 2.0 ** -24, "a near tie would make the comparison moot"
    np.testing.assert_allclose(p["codebooks"], cb, rtol=1e-5, atol=1e-6)
    # tables of the GPU build, sorted, against the oracle's on the same codebooks
    sv, perm = idx.tables_device(torch.from_numpy(Q).cuda())
    torch.cuda.synchronize()
    sv, perm = sv.cpu().numpy().astype(np.float64), perm.cpu().numpy()
    for i in range(len(Q)):
        op, osv = oracle.sort_tables(oracle.tables(Q[i], p["codebooks"]))
        np.testing.assert_allclose(sv[i], osv, rtol=1e-5)
        for s in range(P):
            gap = np.diff(osv[s]) > 1e-5 * osv[s][1:]
            alone = np.concatenate([[gap[0]], gap[:-1] & gap[1:], [gap[-1]]])
            assert (perm[i, s] == op[s])[alone].all()
    # bridge graph from the oracle's codebooks
    gb = _index_cls().build(X, 6, P, K, iters, seed, t, b, codebooks=cb).export()
    off, ids, _ = oracle.bridge_graph(X, cb, t, b)
    ys = literal.all_bridges(cb).astype(np.float64)
    Xd = X.astype(np.float64)
    D = (Xd ** 2).sum(1)[:, None] + (ys ** 2).sum(1)[None] - 2 * Xd @ ys.T     # fp64, every vector to every bridge
    kth = np.sort(D, axis=1)[:, t - 1]                                          # each vector's t-th bridge distance
    goff = gb["bridge_off"].astype(np.int64)
    gids = gb["bridge_ids"].astype(np.int64)
    nb = K ** P
    differ = 0
    for lid in range(nb):
        g = gids[goff[lid]:goff[lid + 1]]
        o = ids[off[lid]:off[lid + 1]].astype(np.int64)
        if np.array_equal(g, o):
            continue
        differ += 1
        tol = 1e-5 * max(D[o, lid].max() if len(o) else 0.0, D[g, lid].max() if len(g) else 0.0)
        assert len(g) <= b and (D[g, lid] <= kth[g] * (1 + 1e-5)).all()      # chosen by each listed vector
        assert (np.diff(D[g, lid]) >= -tol).all()                             # ascending up to rounding
        assert len(g) == len(o) and abs(D[g, lid].sum() - D[o, lid].sum()) <= len(g) * tol
    assert differ <= nb // 100, f"{differ} of {nb} bridge lists differ"


# ---------------------------------------------------------------- budgets above 4096 (the serving stream's range)

def test_large_budgets_uneven_k_bit_exact():
    """Per-query budgets in (4096, 8192] with k in {1, 10, 100} on a bridge-heavy
    index (R = 2, four lists of 32 codewords: most of the budget goes to
    bridges, hundreds of thousands are extracted per query and the
    multi-sequence state moves to global slots), against the oracle."""
    w = synth.scaled(synth.WORKLOADS["hog_like_10m_u8"], 20000, nq=24, d=64, components=64)
    X, Q = synth.base_vectors(w), synth.queries(w)
    idx = _index_cls().build(X, 2, 4, 32, 3, 5, 8, 4)      # 1M bridge vectors, about 2% of them linked
    parts = idx.export()
    rng = np.random.default_rng(8192)
    ks = rng.choice([1, 10, 100], size=len(Q)).astype(np.int32)
    Ts = rng.integers(4097, 8193, size=len(Q)).astype(np.int32)
    Ts[0] = 8192
    gi, gd, st = gpu_search(idx, Q, 100, 8192, 64, ks=ks, Ts=Ts, stats=True)
    print(f"[large-budget] evals {st[:, 0].mean():.0f}, bridges extracted {st[:, 4].mean():.0f}, "
          f"moved {int(st[:, 10].sum())}, re-run {int(st[:, 9].sum())}", flush=True)
    assert (st[:, 6] == 0).all()
    assert (st[:, 10] == 1).any()          # global slots in use
    assert (st[:, 0] == Ts).all()          # every budget spent
    assert_search_equal(idx, parts, X, Q, 100, 8192, 64, ks=ks, Ts=Ts)


def test_budgets_across_all_four_classes_bit_exact():
    """Per-query budgets from 64 to 8192 in one launch on an index of four
    subspaces of 16 codewords: four budget classes (up to 512, 2048, 4096
    and above), each with its own visited-set load and multi-sequence state,
    against the oracle (ids, distances and evaluation traces)."""
    w = synth.scaled(synth.WORKLOADS["hog_like_10m_u8"], 20000, nq=24, d=64, components=64)
    X, Q = synth.base_vectors(w), synth.queries(w)
    idx = _index_cls().build(X, 8, 4, 16, 3, 5, 8, 4)
    parts = idx.export()
    rng = np.random.default_rng(4096)
    ks = rng.choice([1, 10, 100], size=len(Q)).astype(np.int32)
    Ts = np.rint(np.exp(rng.uniform(np.log(64), np.log(8192), size=len(Q)))).astype(np.int32)
    Ts[:4] = [300, 1500, 3000, 8192]  # every class holds a query
    gi, gd, st = gpu_search(idx, Q, 100, 8192, 64, ks=ks, Ts=Ts, stats=True)
    print(f"[four-class] budgets {sorted(Ts.tolist())[:3]}..{Ts.max()}, moved {int(st[:, 10].sum())}, "
          f"re-run {int(st[:, 9].sum())}", flush=True)
    assert (st[:, 6] == 0).all()
    assert_search_equal(idx, parts, X, Q, 100, 8192, 64, ks=ks, Ts=Ts)


def test_one_budget_above_4096_for_more_queries_than_fit_sampled():
    """One budget above 4096 for more queries than the chip holds at the
    larger multi-sequence state: the launch takes the residency-first state;
    sampled queries against the oracle."""
    w = synth.scaled(synth.WORKLOADS["sift_like_1m_u8"], 20000, nq=2000, d=64, components=64)
    X, Q = synth.base_vectors(w), synth.queries(w)
    idx = _index_cls().build(X, 8, 4, 16, 3, 5, 8, 4)
    parts = idx.export()
    T = 6000
    gi, gd, st = gpu_search(idx, Q, 10, T, 64, stats=True)
    assert (st[:, 6] == 0).all()
    rows = np.random.default_rng(6000).choice(len(Q), 12, replace=False)
    print(f"[one-budget] {len(Q)} queries at T={T}, moved {int(st[:, 10].sum())}, re-run {int(st[:, 9].sum())}; "
          f"oracle on rows {rows.tolist()}", flush=True)
    oi, od = oracle.search(X, parts["codebooks"], parts["graph"], parts["bridge_off"], parts["bridge_ids"], Q[rows],
                           10, T, 64)
    np.testing.assert_array_equal(gi[rows], oi)
    np.testing.assert_array_equal(gd[rows].astype(np.float64), np.where(np.isinf(od), 2147483647.0, od))


def test_budget_beyond_lds_uses_a_visited_bitmap_bit_exact():
    """Budgets whose visited set does not fit a workgroup's LDS (beyond about
    31,000 evaluations) keep it as a bitmap over the vectors in global
    memory: per-query budgets on both sides of the limit in one launch,
    bit-exact against the oracle (ids, distances and traces)."""
    w = synth.scaled(synth.WORKLOADS["sift_like_1m_u8"], 50000, nq=8, d=64, components=64)
    X, Q = synth.base_vectors(w), synth.queries(w)
    idx = _index_cls().build(X, 8, 4, 16, 3, 5, 8, 4)
    parts = idx.export()
    ks = np.array([10, 100, 1, 10, 10, 100, 10, 1], np.int32)
    Ts = np.array([40000, 36000, 1000, 33000, 40000, 20000, 512, 40000], np.int32)
    gi, gd, st = gpu_search(idx, Q, 100, 40000, 64, ks=ks, Ts=Ts, stats=True)
    assert (st[:, 6] == 0).all() and (st[:, 0] <= Ts).all()
    print(f"[bitmap] evaluations {st[:, 0].tolist()}", flush=True)
    assert_search_equal(idx, parts, X, Q, 100, 40000, 64, ks=ks, Ts=Ts)


def test_exhaustive_budget_of_a_million_on_a_small_index():
    """A budget of 2^20 on 1,000 vectors: the bitmap set, every reachable
    vector evaluated, the same results as the oracle."""
    w = synth.scaled(synth.WORKLOADS["tiny_10k_u8"], 1000, nq=4)
    X, Q = synth.base_vectors(w), synth.queries(w)
    idx = _index_cls().build(X, 4, 2, 4, 2, 1, 1, 0)
    parts = idx.export()
    assert_search_equal(idx, parts, X, Q, 10, 1 << 20, 64)


# ---------------------------------------------------------------- neighborhood-graph search without bridges

@pytest.mark.parametrize("nseeds,T,L", [(1, 256, 64), (16, 500, 64), (70, 300, 8), (3, 0, 64), (0, 50, 64)])
def test_graph_search_without_bridges_bit_exact(tiny, nseeds, T, L):
    X, Q, p = tiny["X"], tiny["Q"], tiny["parts"]
    seeds = (np.arange(nseeds, dtype=np.int64) * 7919 % len(X)).astype(np.int32)
    if nseeds > 2:
        seeds[-1] = seeds[0]                # a repeated seed is measured once
    qd = torch.from_numpy(Q).cuda()
    tr = torch.empty((len(Q), max(T, 1)), dtype=torch.int32, device="cuda")
    ids, dd = tiny["idx"].search_graph_device(qd, 10, T, torch.from_numpy(seeds).cuda(), queue_len=L, trace=tr)
    torch.cuda.synchronize()
    oi, od, ot = oracle.search(X, p["codebooks"], p["graph"], p["bridge_off"], p["bridge_ids"], Q, 10, T, L,
                               trace_len=max(T, 1), seeds=seeds.astype(np.uint32))
    np.testing.assert_array_equal(ids.cpu().numpy(), oi)
    np.testing.assert_array_equal(dd.cpu().numpy().astype(np.float64), np.where(np.isinf(od), 2147483647.0, od))
    if T > 0:
        np.testing.assert_array_equal(tr.cpu().numpy(), ot)
