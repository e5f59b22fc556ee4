"""Launch settings never change results: look-ahead width, persistent grid,
resident waves per CU and serving order (u8, bit-exact against the oracle and
against each other).  The allocation-free launch replays from a HIP graph."""
import numpy as np
import pytest

import oracle
from paper_1312_3062_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    from paper_1312_3062_amd import Index
    w = synth.scaled(synth.WORKLOADS["sift_like_1m_u8"], 20_000, nq=300, K=12, components=32)
    X, Q = synth.base_vectors(w), synth.queries(w)
    idx = Index.build(X, 16, 4, 12, 5, 77, 20, 5)
    parts = idx.export()
    rng = np.random.default_rng(3)
    ks = rng.choice([1, 10, 100], size=len(Q)).astype(np.int32)
    Ts = np.rint(np.exp(rng.uniform(np.log(8), np.log(1500), size=len(Q)))).astype(np.int32)
    Ts[:5] = 0
    return dict(X=X, Q=Q, idx=idx, parts=parts, ks=ks, Ts=Ts)


def run(small, tune, uneven=True):
    idx, Q = small["idx"], small["Q"]
    qd = torch.from_numpy(Q).cuda()
    kd = torch.from_numpy(small["ks"]).cuda() if uneven else None
    td = torch.from_numpy(small["Ts"]).cuda() if uneven else None
    ids, dd = idx.search_device(qd, 100, 1500, ks=kd, budgets=td, tune=tune)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), dd.cpu().numpy()


def test_uneven_batch_matches_oracle(small):
    gi, gd = run(small, None)
    p = small["parts"]
    oi, od = oracle.search(small["X"], p["codebooks"], p["graph"], p["bridge_off"], p["bridge_ids"], small["Q"],
                           small["ks"], small["Ts"], 64)
    np.testing.assert_array_equal(gi, oi)
    np.testing.assert_array_equal(gd.astype(np.float64), np.where(np.isinf(od), 2147483647.0, od))


@pytest.mark.parametrize("tune", [
    dict(lookahead=1), dict(lookahead=2), dict(lookahead=3),
    dict(persistent=1), dict(persistent=1, waves_per_cu=1), dict(persistent=1, waves_per_cu=3, lookahead=2),
    dict(persistent=1, order=1), dict(persistent=1, order=1, waves_per_cu=2, lookahead=1),
])
def test_launch_settings_do_not_change_results(small, tune):
    base = run(small, None)
    got = run(small, tune)
    np.testing.assert_array_equal(got[0], base[0])
    np.testing.assert_array_equal(got[1], base[1])


def test_autotune_returns_an_equivalent_setting(small):
    idx, Q = small["idx"], small["Q"]
    qd = torch.from_numpy(Q).cuda()
    kd = torch.from_numpy(small["ks"]).cuda()
    td = torch.from_numpy(small["Ts"]).cuda()
    tune = idx.autotune(qd, 100, 1500, ks=kd, budgets=td)
    assert set(tune) == {"lookahead", "persistent", "waves_per_cu", "order"}
    got = run(small, tune)
    base = run(small, None)
    np.testing.assert_array_equal(got[0], base[0])


@pytest.mark.parametrize("tune", [None, dict(persistent=1, order=1)])
def test_workspace_launch_replays_from_a_graph(small, tune):
    idx, Q = small["idx"], small["Q"]
    qd = torch.from_numpy(Q).cuda()
    kd = torch.from_numpy(small["ks"]).cuda()
    td = torch.from_numpy(small["Ts"]).cuda()
    nq = len(Q)
    ws = torch.empty(idx.workspace_bytes(nq, 100, 1500, tune=tune), dtype=torch.uint8, device="cuda")
    out = (torch.empty((nq, 100), dtype=torch.int32, device="cuda"),
           torch.empty((nq, 100), dtype=torch.int32, device="cuda"))
    eager_ids, eager_d = run(small, None)
    # warm up on a side stream, then capture
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        idx.search_device(qd, 100, 1500, ks=kd, budgets=td, out=out, tune=tune, workspace=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        idx.search_device(qd, 100, 1500, ks=kd, budgets=td, out=out, tune=tune, workspace=ws)
    for rep in range(4):
        out[0].fill_(-7)
        out[1].fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out[0].cpu().numpy(), eager_ids, err_msg=f"replay {rep}")
        np.testing.assert_array_equal(out[1].cpu().numpy(), eager_d, err_msg=f"replay {rep}")
        # eager work of the program between replays
        run(small, dict(lookahead=1))
