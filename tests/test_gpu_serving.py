"""Served (continuous batching) results equal plain per-request results, the
result of each query searched alone, and the oracle: a query's result never
depends on what it is batched with."""
import numpy as np
import pytest

import oracle
from paper_1312_3062_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_served_equals_plain_equals_alone():
    from paper_1312_3062_amd import Index
    from paper_1312_3062_amd.serve import Server
    w = synth.scaled(synth.WORKLOADS["sift_like_1m_u8"], 15_000, nq=64, K=10, components=24)
    X = synth.base_vectors(w)
    idx = Index.build(X, 16, 4, 10, 4, 5, 10, 5)
    pool = synth.queries(w, nq=3000)
    reqs = synth.request_stream(w, 3000, rate_rps=4000.0, max_batch=64)[:60]
    for r in reqs:  # keep the oracle check cheap
        r.budget = min(r.budget, 1024)
    srv = Server(idx, w.d, "u8", slots=3, slot_queries=256, kmax=100, queue_len=64)
    a = srv.run_served(reqs, pool, keep_ids=True)
    b = srv.run_plain(reqs, pool, keep_ids=True)
    np.testing.assert_array_equal(a.ids, b.ids)
    assert a.launches < len(reqs)  # requests were batched together
    parts = idx.export()
    row = 0
    for r in reqs[:25]:
        q = pool[r.first:r.first + r.batch]
        ids, _ = idx.search(q, r.k, r.budget)
        np.testing.assert_array_equal(a.ids[row:row + r.batch, :r.k], ids)
        oi, _ = oracle.search(X, parts["codebooks"], parts["graph"], parts["bridge_off"], parts["bridge_ids"], q,
                              r.k, r.budget, 64)
        np.testing.assert_array_equal(ids, oi)
        assert (a.ids[row:row + r.batch, r.k:] == -1).all()
        row += r.batch
    assert (a.latencies_s > 0).all() and (b.latencies_s > 0).all()
