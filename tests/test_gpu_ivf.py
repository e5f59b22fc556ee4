"""Graph-D-ADC (Sec. 5) on the GPU against the oracle, step by step on the
parts the library exports: the vocabulary is the seeded sample; each vector
sits in the list that the oracle's graph search over the centres returns
(bit-exact); lists hold their vectors in increasing id; residual codebooks
after zero and one k-means iteration equal the oracle's up to fp32
rounding of the mean; each code is the fp64-nearest codeword wherever the
nearest is clear of fp32 rounding; and the re-ranked lists match the
oracle's fp64 asymmetric distances (within 1e-4 relative, ids equal except
between candidates whose distances tie within that bound)."""
import numpy as np
import pytest

import oracle
from paper_1312_3062_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SEED = 7
CENTRE_BUDGET = 256
ASSIGN_BUDGET = 128
RTOL = 1e-4


def _build(X, lists, m, iters, seed=SEED):
    from paper_1312_3062_amd.ivf import Ivf
    return Ivf.build(X, lists=lists, pq_m=m, pq_iters=iters, assign_budget=ASSIGN_BUDGET, seed=seed, graph_k=16,
                     P=2, K=16, kmeans_iters=4, bridge_t=1, bridge_b=5, centre_seed=1)


def _assignment(parts, n):
    a = np.full(n, -1, np.int64)
    off, ids = parts["list_off"].astype(np.int64), parts["list_ids"].astype(np.int64)
    for j in range(len(off) - 1):
        a[ids[off[j]:off[j + 1]]] = j
    return a


def _oracle_lists(ivf, Q, W, T):
    """The lists the oracle's graph search over the centres returns."""
    cp = ivf.centres_index().export()
    centres = ivf.export()["centres"]
    lids, _ = oracle.search(centres, cp["codebooks"], cp["graph"], cp["bridge_off"], cp["bridge_ids"], Q, W, T, 64)
    return lids


@pytest.fixture(scope="module")
def data():
    w = synth.scaled(synth.WORKLOADS["sift_like_1m_u8"], 20_000, nq=48)
    return synth.base_vectors(w), synth.queries(w)


@pytest.fixture(scope="module", params=[8, 16], ids=["m8", "m16"])
def built(request, data):
    X, Q = data
    m = request.param
    ivf = _build(X, 256, m, 4)
    parts = ivf.export()
    print(f"[ivf] built m={m}: {ivf.info}", flush=True)
    return dict(X=X, Q=Q, m=m, ivf=ivf, parts=parts, assign=_assignment(parts, len(X)))


def test_vocabulary_and_lists(built):
    X, parts, a = built["X"], built["parts"], built["assign"]
    np.testing.assert_array_equal(parts["centres"], X[oracle.init_rows(len(X), 256, SEED)])
    assert (a >= 0).all()
    off, ids = parts["list_off"], parts["list_ids"]
    assert off[0] == 0 and off[-1] == len(X)
    for j in range(len(off) - 1):
        assert (np.diff(ids[off[j]:off[j + 1]].astype(np.int64)) > 0).all()
    # each vector in the list of the centre the oracle's search returns for it (k = 1)
    ivf = built["ivf"]
    cp = ivf.centres_index().export()
    lids, _ = oracle.search(parts["centres"], cp["codebooks"], cp["graph"], cp["bridge_off"], cp["bridge_ids"], X,
                            1, ASSIGN_BUDGET, 64)
    np.testing.assert_array_equal(a, lids[:, 0])


def test_codes_are_the_nearest_codewords(built):
    X, parts, a, m = built["X"], built["parts"], built["assign"], built["m"]
    R = X.astype(np.float64) - parts["centres"][a].astype(np.float64)
    want, gap = oracle.pq_encode(R, parts["pq"], want_gap=True)
    got = np.empty_like(want)
    got[parts["list_ids"].astype(np.int64)] = parts["codes"]
    ds = X.shape[1] // m
    cb = parts["pq"].astype(np.float64)
    diff = np.argwhere(got != want)
    for i, p in diff:
        sub = R[i, p * ds:(p + 1) * ds]
        dg = ((sub - cb[p, got[i, p]]) ** 2).sum()
        dw = ((sub - cb[p, want[i, p]]) ** 2).sum()
        # fp32 sums of ds squares: only a near tie may go the other way
        assert dg - dw <= 1e-5 * (1.0 + dw), (i, p, dg, dw)
    clear = gap > 1e-5 * (1.0 + gap)
    assert (got[clear] == want[clear]).mean() > 0.9999
    print(f"[ivf] codes differing from the fp64 nearest (near ties): {len(diff)} of {got.size}", flush=True)


@pytest.mark.parametrize("iters", [0, 1])
def test_residual_codebooks_against_the_oracle_kmeans(data, iters):
    X, _ = data
    X = X[:6000]
    m = 8
    ivf = _build(X, 64, m, iters)
    parts = ivf.export()
    a = _assignment(parts, len(X))
    R = (X.astype(np.int64) - parts["centres"][a].astype(np.int64)).astype(np.float32)
    want = oracle.kmeans(R, m, 256, iters, SEED + 1)
    # integer residuals: the first assignment is exact; the mean differs by fp32 rounding only
    np.testing.assert_allclose(parts["pq"], want, rtol=4e-7, atol=1e-5)
    ivf.close()


def _check_ranked(gids, gd, oids, od, all_ids, all_d):
    """GPU list against the oracle's: same padding; distances within RTOL;
    every GPU id a candidate whose oracle distance is its GPU distance; ids
    equal except where the oracle's distances tie within the bound."""
    valid = oids >= 0
    np.testing.assert_array_equal(gids >= 0, valid)
    np.testing.assert_allclose(gd[valid], od[valid], rtol=RTOL, atol=RTOL)
    where = {int(i): float(x) for i, x in zip(all_ids, all_d) if i >= 0}
    g = gids[valid]
    assert len(set(g.tolist())) == len(g)
    for i, gid in enumerate(g):
        assert int(gid) in where, gid
        tol = RTOL * max(1.0, od[i])
        assert abs(where[int(gid)] - gd[i]) <= tol
        if gid != oids[i]:
            assert abs(where[int(gid)] - od[i]) <= 2 * tol
    return int((g != oids[valid]).sum())


@pytest.mark.parametrize("W,L,k", [(8, 2_000, 100), (32, 100_000, 100), (1, 50, 10), (64, 5_000, 1024),
                                   (16, 0, 10), (300, 100_000, 10)])
def test_search_against_the_oracle(built, W, L, k):
    ivf, parts, Q = built["ivf"], built["parts"], built["Q"]
    qd = torch.from_numpy(Q).cuda()
    print(f"[ivf] m={built['m']} lists={W} candidates={L} k={k}", flush=True)
    ids, dd = ivf.search_device(qd, k, W, CENTRE_BUDGET, L)
    torch.cuda.synchronize()
    ids, dd = ids.cpu().numpy(), dd.cpu().numpy()
    # the list choice: the centres' search, bit-exact against the oracle's
    lists = _oracle_lists(ivf, Q, W, CENTRE_BUDGET)
    gl, _ = ivf.centres_index().search(Q, W, CENTRE_BUDGET)
    np.testing.assert_array_equal(gl, lists)
    oids, od, cnt = oracle.ivf_adc(Q, parts["centres"], parts["list_off"], parts["list_ids"], parts["codes"],
                                   parts["pq"], lists, L, k, want_count=True)
    full_k = int(max(1, cnt.max()))
    aids, ad = oracle.ivf_adc(Q, parts["centres"], parts["list_off"], parts["list_ids"], parts["codes"],
                              parts["pq"], lists, L, full_k)
    swaps = 0
    for qi in range(len(Q)):
        swaps += _check_ranked(ids[qi], dd[qi], oids[qi], od[qi], aids[qi], ad[qi])
    if L > 0 and W > 1:
        assert cnt.min() > 0
    print(f"[ivf] candidates per query {cnt.mean():.0f}, ids swapped within near ties: {swaps}", flush=True)


def test_bad_arguments_are_rejected(built):
    from paper_1312_3062_amd._abi import AnnError
    ivf, Q = built["ivf"], built["Q"]
    qd = torch.from_numpy(Q).cuda()
    for k, W in ((0, 4), (1025, 4), (10, 0), (10, 1025)):
        with pytest.raises(AnnError):
            ivf.search_device(qd, k, W, CENTRE_BUDGET, 100)
