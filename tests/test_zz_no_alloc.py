"""ann_search_device_noalloc (the search that allocates nothing, its workspace
a buffer compiled into the library) against ann_search_device, called through
the C ABI: bit-exact on two calls in a row, the second with a smaller input,
on a plain index, on one whose queries move their multi-sequence state to
global slots of the workspace and at budgets whose visited bitmaps live in
the workspace; and a request too large for the buffer is rejected with an
error."""
import ctypes as C

import numpy as np
import pytest

from paper_1312_3062_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _call(name, idx, Q, k, T, ks=None, Ts=None, L=64):
    from paper_1312_3062_amd import _abi
    from paper_1312_3062_amd.index import _stream_ptr, _tptr, search_params
    qd = torch.from_numpy(np.ascontiguousarray(Q)).cuda()
    nq = len(Q)
    ids = torch.full((nq, k), -5, dtype=torch.int32, device="cuda")
    dd = torch.full((nq, k), -5, dtype=torch.int32, device="cuda")
    st = torch.zeros((nq, 12), dtype=torch.int32, device="cuda")
    kd = None if ks is None else torch.from_numpy(np.asarray(ks, np.int32)).cuda()
    td = None if Ts is None else torch.from_numpy(np.asarray(Ts, np.int32)).cuda()
    sp = search_params(L)
    rc = getattr(_abi.lib(), name)(idx._h, _tptr(qd), nq, k, T, _tptr(kd), _tptr(td), C.byref(sp), _tptr(ids),
                                   _tptr(dd), _tptr(st), None, _stream_ptr(None))
    torch.cuda.synchronize()
    return rc, ids.cpu().numpy(), dd.cpu().numpy(), st.cpu().numpy()


def _same(idx, Q, k, T, **kw):
    rc, ai, ad, ast = _call("ann_search_device_noalloc", idx, Q, k, T, **kw)
    assert rc == 0
    rc, bi, bd, bst = _call("ann_search_device", idx, Q, k, T, **kw)
    assert rc == 0
    np.testing.assert_array_equal(ai, bi)
    np.testing.assert_array_equal(ad, bd)
    np.testing.assert_array_equal(ast[:, :9], bst[:, :9])
    return ast


def test_noalloc_equals_the_allocating_search_twice():
    from paper_1312_3062_amd import Index
    w = synth.WORKLOADS["tiny_10k_u8"]
    X, Q = synth.base_vectors(w), synth.queries(w)
    idx = Index.build(X, w.graph_k, w.P, w.K, w.kmeans_iters, w.kmeans_seed, w.bridge_t, w.bridge_b)
    print("[noalloc] tiny index, 100 queries at T=256, then 37 at T=100 with per-query k and budget", flush=True)
    _same(idx, Q, 10, 256)
    rng = np.random.default_rng(3)
    _same(idx, Q[:37], 5, 100, ks=rng.integers(1, 6, 37), Ts=rng.integers(0, 101, 37))


def test_noalloc_with_visited_bitmaps_twice():
    """Budgets beyond LDS: the visited bitmaps live in the buffer too."""
    from paper_1312_3062_amd import Index
    w = synth.scaled(synth.WORKLOADS["sift_like_1m_u8"], 50000, nq=8, d=64, components=64)
    X, Q = synth.base_vectors(w), synth.queries(w)
    idx = Index.build(X, 8, 4, 16, 3, 5, 8, 4)
    print("[noalloc] 8 queries at T=40000, then 3 at T=36000", flush=True)
    _same(idx, Q, 10, 40000)
    _same(idx, Q[:3], 10, 36000)


def test_noalloc_with_global_slots_twice():
    from paper_1312_3062_amd import Index
    rng = np.random.default_rng(77)
    X = rng.integers(0, 256, size=(2000, 32)).astype(np.uint8)
    Q = rng.integers(0, 256, size=(12, 32)).astype(np.uint8)
    idx = Index.build(X, 1, 4, 16, 2, 5, 3, 1)    # lists of one: the enumeration outgrows LDS
    print("[noalloc] bridge-heavy index, 12 queries at T=1800, then 5 at T=900", flush=True)
    st = _same(idx, Q, 10, 1800)
    assert (st[:, 10] == 1).any()                 # global slots of the fixed buffer in use
    _same(idx, Q[:5], 7, 900)


def test_noalloc_rejects_a_request_larger_than_its_buffer():
    from paper_1312_3062_amd import Index, _abi
    rng = np.random.default_rng(5)
    X = rng.integers(0, 256, size=(500, 16)).astype(np.uint8)
    idx = Index.build(X, 4, 2, 4, 2, 1, 1, 0)
    nq = 9_000_000                                # 8 bytes of lists per query: 72 MB > 64 MiB
    print(f"[noalloc] rejection: {nq} queries", flush=True)
    Q = np.zeros((nq, 16), np.uint8)
    rc, _, _, _ = _call("ann_search_device_noalloc", idx, Q, 1, 4)
    assert rc == _abi.ANN_EINVAL
    assert b"workspace" in _abi.lib().ann_last_error()
