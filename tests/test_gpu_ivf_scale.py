"""Graph-D-ADC at the size the benchmark times (1M x 128, 6,144 lists,
16-byte codes, 922 lists and 100,000 candidates a query, centre budget
3,688), on sampled queries against the oracle: the lists bit-exact, the
re-ranked top 100 within 1e-4 of the oracle's fp64 asymmetric distances, ids
equal except between candidates that tie within that bound; and the
vocabulary and a sample of the assignment bit-exact."""
import numpy as np
import pytest

import oracle
from paper_1312_3062_amd import synth
from tests.test_gpu_ivf import _check_ranked

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LISTS, M, SEED = 6144, 16, 7
W, TC, L, K = 922, 3688, 100_000, 100


@pytest.fixture(scope="module")
def full():
    from paper_1312_3062_amd.ivf import Ivf
    w = synth.WORKLOADS["sift_like_1m_u8"]
    X, Q = synth.base_vectors(w), synth.queries(w)
    ivf = Ivf.build(X, lists=LISTS, pq_m=M, pq_iters=4, assign_budget=256, seed=SEED, graph_k=16, P=2, K=16,
                    kmeans_iters=4, bridge_t=1, bridge_b=0, centre_seed=SEED)
    print(f"[ivf-scale] built: {ivf.info}", flush=True)
    return dict(X=X, Q=Q, ivf=ivf, parts=ivf.export(), cparts=ivf.centres_index().export())


def test_vocabulary_and_sampled_assignment(full):
    X, parts, cp = full["X"], full["parts"], full["cparts"]
    np.testing.assert_array_equal(parts["centres"], X[oracle.init_rows(len(X), LISTS, SEED)])
    rows = np.random.default_rng(1).choice(len(X), 2000, replace=False)
    lids, _ = oracle.search(parts["centres"], cp["codebooks"], cp["graph"], cp["bridge_off"], cp["bridge_ids"],
                            X[rows], 1, 256, 64)
    owner = np.empty(len(X), np.int64)
    off = parts["list_off"].astype(np.int64)
    owner[parts["list_ids"].astype(np.int64)] = np.repeat(np.arange(LISTS), np.diff(off))
    np.testing.assert_array_equal(owner[rows], lids[:, 0])


def test_sampled_queries_against_the_oracle(full):
    Q, ivf, parts, cp = full["Q"], full["ivf"], full["parts"], full["cparts"]
    qd = torch.from_numpy(Q).cuda()
    ids, dd = ivf.search_device(qd, K, W, TC, L)
    torch.cuda.synchronize()
    ids, dd = ids.cpu().numpy(), dd.cpu().numpy()
    rows = np.random.default_rng(2).choice(len(Q), 16, replace=False)
    print(f"[ivf-scale] 10K queries searched; oracle on rows {rows.tolist()}", flush=True)
    q = Q[rows]
    lists, _ = oracle.search(parts["centres"], cp["codebooks"], cp["graph"], cp["bridge_off"], cp["bridge_ids"], q,
                             W, TC, 64)
    gl, _ = ivf.centres_index().search(q, W, TC)
    np.testing.assert_array_equal(gl, lists)
    oids, od, cnt = oracle.ivf_adc(q, parts["centres"], parts["list_off"], parts["list_ids"], parts["codes"],
                                   parts["pq"], lists, L, K, want_count=True)
    assert (cnt == L).all()
    aids, ad = oracle.ivf_adc(q, parts["centres"], parts["list_off"], parts["list_ids"], parts["codes"],
                              parts["pq"], lists, L, L)
    swaps = sum(_check_ranked(ids[r], dd[r], oids[i], od[i], aids[i], ad[i]) for i, r in enumerate(rows))
    print(f"[ivf-scale] ids swapped within near ties: {swaps} of {len(rows) * K}", flush=True)
