"""The 1M x 384 fp32 GIST-like workload at full size.  fp32 search against the
oracle (fp64 arithmetic): returned distances within 1e-4 relative of fp64 and
recall@10 within 0.002 of the oracle's; bf16 gather with fp32 re-rank against
the oracle's bf16 form to the same bar; sampled kNN rows equal to the
oracle's up to fp32 rounding of near ties."""
import numpy as np
import pytest

import oracle
from paper_1312_3062_amd import recall_at, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

T = 1024


@pytest.fixture(scope="module")
def gist():
    from paper_1312_3062_amd import Index, knn_device
    w = synth.WORKLOADS["gist_like_1m_f32"]
    X, Q = synth.base_vectors(w), synth.queries(w)
    idx = Index.build(X, w.graph_k, w.P, w.K, w.kmeans_iters, w.kmeans_seed, w.bridge_t, w.bridge_b)
    print(f"[scale-f32] built {w.name}: {idx.info}", flush=True)
    rows = np.random.default_rng(11).choice(len(Q), 200, replace=False)
    # exact top-10 with fp64 distances: 32 candidates of the fp32 scan re-ranked in fp64
    xd = torch.from_numpy(X).cuda()
    cand, _ = knn_device(xd, torch.from_numpy(Q[rows]).cuda(), 32)
    torch.cuda.synchronize()
    cand = cand.cpu().numpy()
    del xd
    gt = np.empty((len(rows), 10), np.int32)
    for i, qi in enumerate(rows):
        d = ((X[cand[i]].astype(np.float64) - Q[qi].astype(np.float64)) ** 2).sum(1)
        gt[i] = cand[i][np.lexsort((cand[i], d))[:10]]
    return dict(w=w, X=X, Q=Q, idx=idx, parts=idx.export(), rows=rows, gt=gt)


def _search(g, **kw):
    qd = torch.from_numpy(g["Q"]).cuda()
    ids, dd = g["idx"].search_device(qd, 10, T, queue_len=g["w"].queue_len, **kw)
    torch.cuda.synchronize()
    return ids.cpu().numpy()[g["rows"]], dd.cpu().numpy()[g["rows"]].astype(np.float64)


def _exact(g, ids):
    Q = g["Q"][g["rows"]].astype(np.float64)
    return ((g["X"][ids].astype(np.float64) - Q[:, None, :]) ** 2).sum(2)


def test_fp32_search_within_tolerance_of_the_oracle(gist):
    p = gist["parts"]
    gi, gd = _search(gist)
    np.testing.assert_allclose(gd, _exact(gist, gi), rtol=1e-4)
    oi, od = oracle.search(gist["X"], p["codebooks"], p["graph"], p["bridge_off"], p["bridge_ids"],
                           gist["Q"][gist["rows"]], 10, T, gist["w"].queue_len)
    rg, ro = recall_at(gi, gist["gt"], 10), recall_at(oi, gist["gt"], 10)
    print(f"[scale-f32] recall@10 gpu {rg:.4f} oracle {ro:.4f}; ids equal in "
          f"{int((gi == oi).all(1).sum())} of {len(gi)} queries", flush=True)
    assert abs(rg - ro) <= 0.002 + 1e-12


def test_bf16_gather_with_fp32_rerank_against_the_oracle(gist):
    """bf16 rows drive the traversal, the best rerank_k are re-ranked on the
    fp32 rows: against the oracle's bf16 form (rows rounded to nearest even,
    fp64 arithmetic) on the same index, returned distances within 1e-4
    relative of fp64 and recall@10 within 0.002 of the oracle's."""
    p = gist["parts"]
    bi, bd = _search(gist, precision=1, rerank_k=40)
    np.testing.assert_allclose(bd, _exact(gist, bi), rtol=1e-4)
    assert (np.diff(bd, axis=1) >= 0).all()
    oi, od = oracle.search(gist["X"], p["codebooks"], p["graph"], p["bridge_off"], p["bridge_ids"],
                           gist["Q"][gist["rows"]], 10, T, gist["w"].queue_len, precision=1, rerank_k=40)
    rb, ro = recall_at(bi, gist["gt"], 10), recall_at(oi, gist["gt"], 10)
    print(f"[scale-f32] bf16+rerank recall@10 gpu {rb:.4f} oracle {ro:.4f}; ids equal in "
          f"{int((bi == oi).all(1).sum())} of {len(bi)} queries", flush=True)
    assert abs(rb - ro) <= 0.002 + 1e-12
    same = (bi == oi).all(1)
    np.testing.assert_allclose(bd[same], od[same], rtol=1e-4)


def test_sampled_knn_rows_up_to_rounding(gist):
    X, p = gist["X"], gist["parts"]
    rows = np.unique(np.concatenate([[0, len(X) - 1], np.random.default_rng(12).choice(len(X), 14, replace=False)]))
    oi, od = oracle.knn_graph_rows(X, rows, gist["w"].graph_k)
    g = p["graph"][rows].astype(np.int64)
    gd = ((X[g].astype(np.float64) - X[rows].astype(np.float64)[:, None, :]) ** 2).sum(2)
    np.testing.assert_allclose(gd, od, rtol=1e-5)   # the same distances in the same order
    assert (g != rows[:, None]).all()
    same = (g == oi).mean()
    assert same >= 0.97, f"only {same:.3f} of the sampled graph entries agree"
