"""The library's request server (continuous batching, admission by footprint)
against plain per-request launches, each query searched alone, and the
oracle: a query's result never depends on what it is batched with, and the
server finishes every request whatever its memory and LDS limits."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_1312_3062_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    from paper_1312_3062_amd import Index
    w = synth.scaled(synth.WORKLOADS["sift_like_1m_u8"], 15_000, nq=64, K=10, components=24)
    X = synth.base_vectors(w)
    idx = Index.build(X, 16, 4, 10, 4, 5, 10, 5)
    pool = synth.queries(w, nq=4000)
    return dict(w=w, X=X, idx=idx, pool=pool, parts=idx.export())


def test_served_equals_plain_equals_alone(small):
    from paper_1312_3062_amd.serve import Server
    w, X, idx, pool = small["w"], small["X"], small["idx"], small["pool"]
    reqs = synth.request_stream(w, 3000, rate_rps=4000.0, max_batch=64)[:60]
    for r in reqs:  # keep the oracle check cheap
        r.budget = min(r.budget, 1024)
    srv = Server(idx, w.d, "u8", slots=3, slot_queries=256, kmax=100, max_budget=1024, queue_len=64)
    print("[serving] 60 requests, budgets <= 1024", flush=True)
    a = srv.run_served(reqs, pool, keep_ids=True)
    b = srv.run_plain(reqs, pool, keep_ids=True)
    np.testing.assert_array_equal(a.ids, b.ids)
    assert a.launches < len(reqs)  # requests were batched together
    parts = small["parts"]
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
    srv.close()


def test_tight_footprint_limits_serve_every_request_the_same(small):
    """An arena of one full micro-batch and LDS for a single resident round:
    requests wait for memory and LDS to free up, and still come back
    identical to the plain launches, budgets up to 8192 included."""
    from paper_1312_3062_amd.serve import Server
    w, idx, pool = small["w"], small["idx"], small["pool"]
    reqs = synth.request_stream(w, 4000, rate_rps=20000.0, max_batch=128, seed_offset=3)[:80]
    roomy = Server(idx, w.d, "u8", slots=4, slot_queries=256, kmax=100, max_budget=8192)
    one = roomy.footprint(256, 100, 8192)["device_bytes"]
    tight = Server(idx, w.d, "u8", slots=4, slot_queries=256, kmax=100, max_budget=8192, device_bytes=one,
                   lds_rounds=1)
    print(f"[serving] 80 requests through an arena of {one} bytes", flush=True)
    a = tight.run_served(reqs, pool, keep_ids=True)
    b = roomy.run_served(reqs, pool, keep_ids=True)
    c = roomy.run_plain(reqs, pool, keep_ids=True)
    np.testing.assert_array_equal(a.ids, c.ids)
    np.testing.assert_array_equal(b.ids, c.ids)
    inf = tight.info()
    assert inf["pending"] == 0 and inf["busy_slots"] == 0 and inf["device_in_flight"] == 0
    assert inf["lds_in_flight"] == 0
    fp = tight.footprint(10, 10, 8192)
    assert fp["lds_bytes"] > tight.footprint(10, 10, 512)["lds_bytes"] > 0
    tight.close()
    roomy.close()


def test_server_rejects_requests_it_cannot_serve(small):
    from paper_1312_3062_amd import _abi
    from paper_1312_3062_amd.serve import Server
    w, idx, pool = small["w"], small["idx"], small["pool"]
    srv = Server(idx, w.d, "u8", slots=2, slot_queries=64, kmax=10, max_budget=512)
    L = _abi.lib()
    t = C.c_int64()
    q = np.ascontiguousarray(pool[:100])
    for nq, k, T in ((65, 10, 100), (10, 11, 100), (10, 10, 513), (0, 10, 100)):
        rc = L.ann_server_submit(srv._h, q.ctypes.data_as(C.c_void_p), nq, k, T, C.byref(t))
        assert rc == _abi.ANN_EINVAL, (nq, k, T)
    assert L.ann_server_submit(srv._h, q.ctypes.data_as(C.c_void_p), 5, 10, 100, C.byref(t)) == 0
    assert L.ann_server_drain(srv._h) == 0
    ids = np.empty((5, 10), np.int32)
    dd = np.empty((5, 10), np.int32)
    assert L.ann_server_result(srv._h, t.value, ids.ctypes.data_as(C.c_void_p), dd.ctypes.data_as(C.c_void_p)) == 0
    ref, refd = idx.search(q[:5], 10, 100)
    np.testing.assert_array_equal(ids, ref)
    np.testing.assert_array_equal(dd, refd)
    assert L.ann_server_result(srv._h, t.value, ids.ctypes.data_as(C.c_void_p),
                               dd.ctypes.data_as(C.c_void_p)) == _abi.ANN_EINVAL   # released
    srv.close()
