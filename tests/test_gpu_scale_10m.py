"""Parity at the full size of the 10M x 128 u8 workload (K = 64: 16.8M bridge
vectors): an uneven batch of 100K queries with their own k and budget, in one
persistent launch captured in a HIP graph, checked on sampled queries against
the oracle; sampled kNN rows (matrix-core build) against brute force; bridge
lists through the property that fixes them."""
import numpy as np
import pytest

import oracle
from paper_1312_3062_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hog():
    from paper_1312_3062_amd import Index
    w = synth.WORKLOADS["hog_like_10m_u8"]
    X, Q = synth.base_vectors(w), synth.queries(w)
    ks, Ts = synth.per_query_k_budget(w)
    idx = Index.build(X, w.graph_k, w.P, w.K, w.kmeans_iters, w.kmeans_seed, w.bridge_t, w.bridge_b)
    print(f"[scale-10m] built {w.name}: {idx.info}", flush=True)
    return dict(w=w, X=X, Q=Q, ks=ks, Ts=Ts, idx=idx, parts=idx.export())


def test_uneven_batch_in_a_graph_equals_the_oracle(hog):
    w, X, Q, ks, Ts, idx, p = (hog[k] for k in ("w", "X", "Q", "ks", "Ts", "idx", "parts"))
    nq, kmax, tmax = len(Q), int(ks.max()), int(Ts.max())
    qd, kd, td = torch.from_numpy(Q).cuda(), torch.from_numpy(ks).cuda(), torch.from_numpy(Ts).cuda()
    tune = dict(persistent=1, order=1)
    ws = torch.empty(idx.workspace_bytes(nq, kmax, tmax, tune=tune), dtype=torch.uint8, device="cuda")
    out = (torch.empty((nq, kmax), dtype=torch.int32, device="cuda"),
           torch.empty((nq, kmax), dtype=torch.int32, device="cuda"))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        idx.search_device(qd, kmax, tmax, ks=kd, budgets=td, out=out, tune=tune, workspace=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    eager = (out[0].cpu().numpy().copy(), out[1].cpu().numpy().copy())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        idx.search_device(qd, kmax, tmax, ks=kd, budgets=td, out=out, tune=tune, workspace=ws)
    for rep in range(2):
        out[0].fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out[0].cpu().numpy(), eager[0], err_msg=f"replay {rep}")
    rng = np.random.default_rng(21)
    rows = np.sort(np.concatenate([[0, nq - 1], rng.choice(nq, 78, replace=False),
                                   rng.choice(np.nonzero(Ts > 2048)[0], 20, replace=False)]))
    oi, od = oracle.search(X, p["codebooks"], p["graph"], p["bridge_off"], p["bridge_ids"], Q[rows], ks[rows],
                           Ts[rows], w.queue_len)
    np.testing.assert_array_equal(eager[0][rows], oi)
    np.testing.assert_array_equal(eager[1][rows].astype(np.float64), np.where(np.isinf(od), 2147483647.0, od))


def test_sampled_knn_rows_are_exact(hog):
    X, p, w = hog["X"], hog["parts"], hog["w"]
    rows = np.unique(np.concatenate([[0, len(X) - 1], np.random.default_rng(22).choice(len(X), 6, replace=False)]))
    oi, _ = oracle.knn_graph_rows(X, rows, w.graph_k)
    np.testing.assert_array_equal(p["graph"][rows].astype(np.int64), oi.astype(np.int64))


def test_bridge_lists_hold_exactly_the_b_nearest_choosers(hog):
    X, p, w = hog["X"], hog["parts"], hog["w"]
    cb, off, bids = p["codebooks"], p["bridge_off"].astype(np.int64), p["bridge_ids"].astype(np.int64)
    P, K, t, b = w.P, w.K, w.bridge_t, w.bridge_b

    def digits(lid):
        out = []
        for _ in range(P):
            out.append(lid % K)
            lid //= K
        return out[::-1]

    tabs, tops = {}, {}

    def tab(j):
        if j not in tabs:
            tabs[j] = oracle.tables(X[j], cb)
        return tabs[j]

    def top(j):
        if j not in tops:
            tops[j] = set(int(v) for v in oracle.mseq(tab(j), t)[0])
        return tops[j]

    for i in np.random.default_rng(23).choice(len(X), 20, replace=False):
        i = int(i)
        lids, sums, _ = oracle.mseq(tab(i), t)
        for lid, s in zip(lids, sums):
            lid = int(lid)
            lst = bids[off[lid]:off[lid + 1]]
            keys = [(sum(tab(int(j))[q][dg] for q, dg in enumerate(digits(lid))), int(j)) for j in lst]
            assert keys == sorted(keys) and len(lst) <= b
            if i not in set(lst.tolist()):
                assert len(lst) == b and all(kj < (s, i) for kj in keys), f"ref {i} missing from bridge {lid}"
            for j in lst:
                assert lid in top(int(j)), f"ref {int(j)} listed on bridge {lid} it did not choose"
