"""Benchmark: QPS at recall@10 >= 0.9 on 1M x 128 uint8 (SIFT-like synthetic data).

One step = one batched search of all queries (tables, sort, multi-sequence,
traversal) on device-resident inputs.  Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(stats: np.ndarray, d_bytes: int, R: int, k: int, query_bytes: int) -> np.ndarray:
    """Bytes the method must move per query, from the kernel's own counters:
    gathered rows + kNN rows of expanded references + two CSR offsets per
    extracted bridge + bridge-list ids + query in + results out."""
    evals = stats[:, 0].astype(np.int64)
    rpop = stats[:, 1].astype(np.int64)
    bids = stats[:, 3].astype(np.int64)
    bgen = stats[:, 4].astype(np.int64)
    return evals * d_bytes + rpop * 4 * R + bgen * 8 + bids * 4 + query_bytes + 8 * k


def gt_f32(X, xd, Q, k, torch, knn_device, cand=32):
    """Exact k nearest of fp32 data with fp64 distances: the `cand` nearest by
    the GPU's fp32 scan, re-ranked in fp64 by (distance, id).  fp32 rounding
    (relative 1e-6 here) does not move a true top-k vector beyond rank 32
    unless the k-th and 32nd distances lie within that of each other."""
    ids, _ = knn_device(xd, torch.from_numpy(np.ascontiguousarray(Q)).cuda(), cand)
    torch.cuda.synchronize()
    ids = ids.cpu().numpy()
    out = np.empty((len(Q), k), np.int32)
    for i in range(len(Q)):
        d = ((X[ids[i]].astype(np.float64) - Q[i].astype(np.float64)) ** 2).sum(1)
        o = np.lexsort((ids[i], d))[:k]
        out[i] = ids[i][o]
    return out


def _time_modes(idx, w, qd, gt, T, torch, steps):
    """recall@k and kernel time (HIP events) of the fp32 search and of the bf16
    gather with fp32 re-rank on one batch."""
    from paper_1312_3062_amd import recall_at
    out = {}
    for name, prec, rr in (("fp32", 0, 0), ("bf16_rerank", 1, 4 * w.k)):
        ids, _ = idx.search_device(qd, w.k, T, queue_len=w.queue_len, precision=prec, rerank_k=rr)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for a, b in ev:
            a.record()
            idx.search_device(qd, w.k, T, queue_len=w.queue_len, precision=prec, rerank_k=rr)
            b.record()
        torch.cuda.synchronize()
        kms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        out[name] = {"recall@10": round(recall_at(ids.cpu().numpy(), gt, w.k), 4), "kernel_ms": round(kms, 3),
                     "qps": round(qd.shape[0] / (kms * 1e-3), 1)}
    return out


def precision_leg(idx, w, X, Q, gt, T, torch, steps=10, big=None):
    """fp32 search vs bf16 gather with fp32 re-rank on the same queries: recall@k,
    queries/s (kernel time, HIP events) and the error of returned and candidate
    distances against fp64.  `big` = (queries, ground truth): a larger batch of
    the same recipe, timed in both modes (there the gathers, not the slowest
    query, set the launch time).  The larger batch runs first, so the last
    launches of each mode are still those of the queries given."""
    from paper_1312_3062_amd import recall_at
    res_big = None
    if big is not None:
        bq, bgt = big
        res_big = (f"batch_{len(bq)}", _time_modes(idx, w, torch.from_numpy(bq).cuda(), bgt, T, torch, max(3, steps // 2)))
    qd = torch.from_numpy(Q).cuda()
    res = {}
    Xd = X.astype(np.float64)
    Qd = Q.astype(np.float64)
    for name, prec, rr in (("fp32", 0, 0), ("bf16_rerank", 1, 4 * w.k)):
        ids, dd = idx.search_device(qd, w.k, T, queue_len=w.queue_len, precision=prec, rerank_k=rr)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for a, b in ev:
            a.record()
            idx.search_device(qd, w.k, T, queue_len=w.queue_len, precision=prec, rerank_k=rr)
            b.record()
        torch.cuda.synchronize()
        kms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        ids, dd = ids.cpu().numpy(), dd.cpu().numpy().astype(np.float64)
        ex = ((Xd[ids] - Qd[:, None, :]) ** 2).sum(2)
        rel = np.abs(dd - ex) / np.maximum(ex, 1e-30)
        res[name] = {"recall@10": round(recall_at(ids, gt, w.k), 4), "rerank_k": rr or None,
                     "kernel_ms": round(kms, 3), "qps": round(len(Q) / (kms * 1e-3), 1),
                     "max_rel_err_returned": float(f"{rel.max():.3g}"),
                     "mean_rel_err_returned": float(f"{rel.mean():.3g}")}
    # the bf16 approximation the traversal runs on, for the fp32 results' ids
    ids, _ = idx.search_device(qd, w.k, T, queue_len=w.queue_len)
    torch.cuda.synchronize()
    ids = ids.cpu().numpy()
    xb = torch.from_numpy(X[ids.reshape(-1)]).to(torch.bfloat16).to(torch.float64).numpy().reshape(ids.shape + (-1,))
    bd = ((xb - Qd[:, None, :]) ** 2).sum(2)
    ex = ((Xd[ids] - Qd[:, None, :]) ** 2).sum(2)
    relb = np.abs(bd - ex) / np.maximum(ex, 1e-30)
    res["bf16_candidate_distance"] = {"max_rel_err": float(f"{relb.max():.3g}"),
                                      "mean_rel_err": float(f"{relb.mean():.3g}"),
                                      "note": "(q - bf16(x))^2 summed in fp64 vs fp64, same ids"}
    if res_big is not None:
        res[res_big[0]] = res_big[1]
    return res


def serving_leg(idx, w, args, gt_fn, fixed_k=None, fixed_budget=None, requests=None):
    """Poisson request streams at fractions of the plain saturation rate, served
    (continuous batching) and plain (one launch per request).  With fixed_k /
    fixed_budget every request uses them (the recall >= 0.9 operating point);
    otherwise k and the budget vary per request."""
    from paper_1312_3062_amd import recall_at, synth
    from paper_1312_3062_amd.serve import Server

    def stream(rate, off):
        rs = synth.request_stream(w, args.serve_pool, rate, seed_offset=off)
        for r in rs:
            if fixed_k:
                r.k = fixed_k
            if fixed_budget:
                r.budget = fixed_budget
        return rs

    pool = synth.queries(w, nq=args.serve_pool)
    srv = Server(idx, w.d, "u8" if w.dtype == "u8" else "f32", slots=4, slot_queries=4096, kmax=100,
                 max_budget=max(8192, fixed_budget or 0), queue_len=w.queue_len)
    probe = stream(1.0, 99)[:200]
    srv.run_served(probe[:20], pool)  # warm-up of both paths
    srv.run_plain(probe[:20], pool)
    svc = srv.plain_service_time(probe, pool)
    sat = 1.0 / svc
    log(f"[serve] plain service time {svc * 1e3:.2f} ms/request -> saturation {sat:.1f} requests/s")
    runs, checks = [], {}
    for i, f in enumerate(args.serve_loads):
        reqs = stream(f * sat, i)[:requests or args.serve_requests]
        keep = i == 1
        a = srv.run_served(reqs, pool, f * sat, keep_ids=keep)
        b = srv.run_plain(reqs, pool, f * sat, keep_ids=keep)
        offered = sum(r.batch for r in reqs) / max(1e-9, reqs[-1].arrival_s - reqs[0].arrival_s)
        for r in (a, b):
            sm = r.summary()
            sm["load"] = f
            sm["offered_qps"] = round(offered, 1)
            runs.append(sm)
            log(f"[serve] load {f:.1f}x {sm['mode']:6s}: {sm['qps']:.0f} QPS, p50 {sm['p50_ms']:.2f} ms, "
                f"p99 {sm['p99_ms']:.2f} ms, {sm['launches']} launches")
        if keep:
            checks["mix_invariant"] = bool(np.array_equal(a.ids, b.ids))
            nq = a.ids.shape[0]
            kq = np.concatenate([[r.k] * r.batch for r in reqs])
            sel = np.nonzero(kq >= 10)[0]
            gt = gt_fn(pool[:nq][sel])
            checks["recall@10_k>=10"] = round(recall_at(a.ids[sel], gt, 10), 4)
            log(f"[serve] same ids served and plain: {checks['mix_invariant']}; "
                f"recall@10 over {len(sel)} queries with k>=10: {checks['recall@10_k>=10']}")
    served = [r for r in runs if r["mode"] == "served"]
    plain = [r for r in runs if r["mode"] == "plain"]
    keeps = lambda r: r["qps"] >= 0.95 * r["offered_qps"]  # noqa: E731  (kept up with the arrivals)
    srv.close()
    return {"index": w.name, "k": fixed_k or "1|10|100", "budget": fixed_budget or "128..8192",
            "requests_per_run": len(reqs), "plain_service_ms": round(svc * 1e3, 3),
            "plain_saturation_rps": round(sat, 2), "runs": runs,
            "served_max_qps": max(r["qps"] for r in served), "plain_max_qps": max(r["qps"] for r in plain),
            "served_keeps_up_to_load": max([r["load"] for r in served if keeps(r)], default=None),
            "plain_keeps_up_to_load": max([r["load"] for r in plain if keeps(r)], default=None), **checks}


def bridge_alpha(idx):
    """The bridge graph's occupancy, from the exported CSR: alpha as in the
    paper's Table 1 (reference vectors linked to some bridge, per bridge
    vector: #linked / K^P) and the share of bridge vectors whose list is not
    empty."""
    parts = idx.export()
    off = np.asarray(parts["bridge_off"], dtype=np.int64)
    nb = max(1, len(off) - 1)
    linked = np.unique(np.asarray(parts["bridge_ids"])[:int(off[-1])]).size
    return {"alpha": linked / nb, "linked": int(linked), "nonempty_share": float(np.count_nonzero(np.diff(off))) / nb}


def uneven_leg(w, args, torch, serve_mixed=False, cpu_baseline=True):
    """The 10M workload: 100K queries with their own k (1, 10, 100) and budget
    (log-uniform 64..4096) searched by one persistent launch captured in a HIP
    graph and replayed; recall@10 over the queries with k >= 10.  With
    serve_mixed, request streams with k in {1, 10, 100} and budgets 128..8192
    on the same index, served and plain.  Returns the figures as a dict."""
    from paper_1312_3062_amd import Index, knn_device, recall_at, synth
    t0 = time.time()
    X = synth.base_vectors(w)
    Q = synth.queries(w)
    ks, Ts = synth.per_query_k_budget(w)
    log(f"[bench] data {X.shape} {X.dtype}, {len(Q)} queries, mean budget {Ts.mean():.0f} in {time.time() - t0:.1f}s")
    torch.cuda.set_device(0)
    t0 = time.time()
    idx = Index.build(X, w.graph_k, w.P, w.K, w.kmeans_iters, w.kmeans_seed, w.bridge_t, w.bridge_b)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    log(f"[bench] index built in {build_s:.1f}s: {idx.info}")
    alpha = bridge_alpha(idx)
    log(f"[bench] bridge graph: {alpha['linked']} reference vectors linked, alpha {alpha['alpha']:.4f}; "
        f"{alpha['nonempty_share']:.4f} of the K^P lists not empty")
    xd = torch.from_numpy(X).cuda()
    qd = torch.from_numpy(Q).cuda()
    gt, _ = knn_device(xd, qd, 10)
    torch.cuda.synchronize()
    gt = gt.cpu().numpy()
    nq, kmax, tmax = len(Q), int(ks.max()), int(Ts.max())
    kd, td = torch.from_numpy(ks).cuda(), torch.from_numpy(Ts).cuda()
    stats = torch.empty((nq, 12), dtype=torch.int32, device="cuda")
    ids, _ = idx.search_device(qd, kmax, tmax, ks=kd, budgets=td, queue_len=w.queue_len, stats=stats)
    torch.cuda.synchronize()
    st = stats.cpu().numpy()
    if (st[:, 6] != 0).any():
        raise RuntimeError(f"{int((st[:, 6] != 0).sum())} queries overflowed a per-query structure")
    ids = ids.cpu().numpy()
    sel = ks >= 10
    rec = recall_at(ids[sel], gt[sel], 10)
    log(f"[bench] recall@10 over {int(sel.sum())} queries with k >= 10: {rec:.4f}; evals {st[:, 0].mean():.0f}, "
        f"bridge pops {st[:, 2].mean():.2f}, moved {int(st[:, 10].sum())}, re-run {int(st[:, 9].sum())}")
    tune = idx.autotune(qd, kmax, tmax, ks=kd, budgets=td, queue_len=w.queue_len)
    log(f"[bench] autotuned launch setting: {tune}")
    ws = torch.empty(idx.workspace_bytes(nq, kmax, tmax, queue_len=w.queue_len, tune=tune), dtype=torch.uint8,
                     device="cuda")
    out = (torch.empty((nq, kmax), dtype=torch.int32, device="cuda"),
           torch.empty((nq, kmax), dtype=torch.int32, device="cuda"))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        idx.search_device(qd, kmax, tmax, ks=kd, budgets=td, queue_len=w.queue_len, out=out, tune=tune, workspace=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        idx.search_device(qd, kmax, tmax, ks=kd, budgets=td, queue_len=w.queue_len, out=out, tune=tune, workspace=ws)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t_wall = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        g.replay()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    kms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    same = bool(np.array_equal(out[0].cpu().numpy(), ids))
    qps = nq * args.steps / wall
    B = algorithmic_bytes(st, X.shape[1], w.graph_k, 0, X.shape[1]) + 8 * ks.astype(np.int64)
    achieved = float(B.sum()) / (kms * 1e-3) / 1e9
    log(f"[bench] graph replay: {kms:.3f} ms per batch, {qps:.0f} QPS, same ids as eager: {same}; "
        f"algorithmic {B.sum() / 1e9:.3f} GB -> {achieved:.1f} GB/s")
    del g, ws, out

    cpu = None
    if cpu_baseline and not args.no_cpu_baseline:
        import oracle
        parts = idx.export()
        m = args.cpu_sample or 4000
        t0 = time.perf_counter()
        oi, _ = oracle.search(X, parts["codebooks"], parts["graph"], parts["bridge_off"], parts["bridge_ids"],
                              Q[:m], ks[:m], Ts[:m], w.queue_len)
        cpu_s = time.perf_counter() - t0
        eq = bool(all(np.array_equal(oi[i, :ks[i]], ids[i, :ks[i]]) for i in range(m)))
        cpu = {"value": round(m / cpu_s, 2), "unit": "queries/s", "cores": 1, "kind": "oracle",
               "sample": f"first {m} of {nq} queries with their own k and budget ({cpu_s:.1f} s), single-threaded "
                         f"C oracle on the GPU-built index; ids identical to the GPU: {eq}", "host": host_info()}
        log(f"[bench] oracle: {m} queries in {cpu_s:.1f}s -> {m / cpu_s:.1f} QPS (ids equal: {eq})")

    serving = None
    if serve_mixed:
        def gt_fn(qs):
            r, _ = knn_device(xd, torch.from_numpy(np.ascontiguousarray(qs)).cuda(), 10)
            torch.cuda.synchronize()
            return r.cpu().numpy()

        serving = serving_leg(idx, w, args, gt_fn, requests=args.serve_requests_10m)
    del xd
    from paper_1312_3062_amd.profiling import read_traffic_record
    trec = read_traffic_record(os.path.join(ROOT, "profiles", f"k_search_{w.name}_traffic.md"))
    traffic = trec["bytes_per_launch"] if trec and trec.get("workload") == f"{w.name} uneven nq={nq}" else None
    return {
        "value": round(qps, 1), "ms_per_step": round(wall * 1000.0 / args.steps, 4),
        "config": {"workload": w.name, "n": w.n, "d": w.d, "queries": nq, "k": "1|10|100",
                   "budget": "log-uniform 64..4096", "mean_budget": round(float(Ts.mean()), 1),
                   "queue_len": w.queue_len, "graph_k": w.graph_k, "P": w.P, "K": w.K, "bridge_t": w.bridge_t,
                   "bridge_b": w.bridge_b, "recall@10_k>=10": round(rec, 4), "launch": tune,
                   "hip_graph": True, "graph_ids_equal_eager": same, "build_s": round(build_s, 2),
                   "bridge_alpha": round(alpha["alpha"], 5), "bridges_nonempty": round(alpha["nonempty_share"], 5)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "kernel": "k_search", "kernel_ms": round(kms, 4), "algorithmic_bytes_per_launch": int(B.sum())},
        "cpu_baseline": cpu,
        "serving": serving,
    }


def copy_probe(torch):
    """bitwise_not over 2^28 int32: reads 1 GiB, writes 1 GiB, no reuse (the
    known traffic that calibrates the hardware counters)."""
    src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.bitwise_not(src, out=dst)
    torch.cuda.synchronize()
    del src, dst
    log("[bench] copy probe: 3 x bitwise_not over 1 GiB")


def bench_uneven(w, args, torch):
    """One JSON line for the 10M workload alone (--workload hog_like_10m_u8)."""
    leg = uneven_leg(w, args, torch, serve_mixed=args.serve_mixed)
    if args.copy_probe:
        copy_probe(torch)
    line = {
        "metric": f"QPS of one uneven batch (k in 1|10|100, budget log-uniform 64..4096), "
                  f"{w.n // 1_000_000}M x{w.d} uint8",
        "value": leg["value"], "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": leg["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic", "config": leg["config"],
        "roofline": leg["roofline"], "cpu_baseline": leg["cpu_baseline"],
        "serving": {"mixed_k_budget": leg["serving"]} if leg["serving"] else None,
    }
    print(json.dumps(line), flush=True)


def bridge_sweep(w, args, torch):
    """The bridge-graph rule and the codebooks (Sec. 4.1, Table 1, Sec. 5.2's
    study of partitions and clusters) on the 1M x 128 data: for P in {2, 4}
    subspaces, several K and the rules (t, b) in {(1, all), (1, 5), (100, 5)},
    the reference vectors linked to bridge vectors (#reference), alpha =
    #reference / K^P, and the search's recall@10 and queries/s at the
    smallest budget on the doubling grid (refined by eighths) that reaches
    recall@10 >= 0.9.  Every index shares the one exact kNN graph."""
    from paper_1312_3062_amd import Index, knn_device, recall_at, synth
    X, Q = synth.base_vectors(w), synth.queries(w)
    torch.cuda.set_device(0)
    base = Index.build(X, w.graph_k, w.P, w.K, w.kmeans_iters, w.kmeans_seed, w.bridge_t, w.bridge_b)
    G = base.export()["graph"]
    del base
    xd, qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    gt, _ = knn_device(xd, qd, w.k)
    torch.cuda.synchronize()
    gt = gt.cpu().numpy()
    del xd
    out = (torch.empty((len(Q), w.k), dtype=torch.int32, device="cuda"),
           torch.empty((len(Q), w.k), dtype=torch.int32, device="cuda"))

    def search(idx, T):
        idx.search_device(qd, w.k, T, queue_len=w.queue_len, out=out)
        torch.cuda.synchronize()
        rec = recall_at(out[0].cpu().numpy(), gt, w.k)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
        for a, b in ev:
            a.record()
            idx.search_device(qd, w.k, T, queue_len=w.queue_len, out=out)
            b.record()
        torch.cuda.synchronize()
        return rec, float(np.median([a.elapsed_time(b) for a, b in ev]))

    rows = []
    for P, K in ((2, 32), (2, 64), (2, 128), (2, 256), (4, 16), (4, 32), (4, 50)):
        for t, b in ((1, 0), (1, 5), (100, 5)):
            t0 = time.time()
            idx = Index.build(X, w.graph_k, P, K, w.kmeans_iters, w.kmeans_seed, t, b, graph=G)
            build_s = time.time() - t0
            al = bridge_alpha(idx)
            fixed = {T: search(idx, T) for T in (512, 1152, 2048)}
            prev, hit = None, None
            T = 128
            while T <= 16384:
                rec, ms = fixed[T] if T in fixed else search(idx, T)
                if rec >= 0.9:
                    hit = (T, rec, ms)
                    break
                prev, T = T, T * 2
            if hit and prev:
                step = max(16, prev // 8)
                for T2 in range(prev + step, hit[0], step):
                    rec, ms = search(idx, T2)
                    if rec >= 0.9:
                        hit = (T2, rec, ms)
                        break
            row = {"P": P, "K": K, "bridges": K ** P, "t": t, "b": b or "all", "reference": al["linked"],
                   "alpha": round(al["alpha"], 5), "lists_nonempty": round(al["nonempty_share"], 5),
                   "recall@10": {str(T): round(v[0], 4) for T, v in fixed.items()},
                   "budget_at_0.9": hit[0] if hit else None,
                   "qps_at_0.9": round(len(Q) / (hit[2] * 1e-3), 1) if hit else None,
                   "build_s": round(build_s, 2)}
            rows.append(row)
            log(f"[sweep] P={P} K={K} t={t} b={b or 'all'}: #reference {al['linked']}, alpha {al['alpha']:.4f}, "
                f"recall@10 at 512/1152/2048 {[row['recall@10'][k] for k in ('512', '1152', '2048')]}, "
                f"T for 0.9: {row['budget_at_0.9']}, QPS {row['qps_at_0.9']}")
            del idx
    best = max((r["qps_at_0.9"] or 0.0) for r in rows)
    line = {"metric": "QPS at recall@10>=0.9 per bridge rule and codebook, 1M x128 uint8", "value": best,
            "unit": "queries/s", "n_gpus": 1, "steps": 3, "warmup": 1, "ms_per_step": None,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
            "config": {"workload": w.name, "n": w.n, "queries": len(Q), "k": w.k, "queue_len": w.queue_len,
                       "graph_k": w.graph_k},
            "bridge_sweep": rows,
            "paper_table_1": {"SIFT 1M, 4 x 50": {"reference": 715000, "alpha": 0.114},
                              "GIST 1M, 4 x 50": {"reference": 599000, "alpha": 0.0959},
                              "HOG 10M, 4 x 100": {"reference": 5730000, "alpha": 0.0573}}}
    print(json.dumps(line), flush=True)


def host_info() -> dict:
    """The host the oracle is timed on: logical CPUs, the ones this process may
    use, the CPU model and whether SMT is on."""
    info = {"nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0)), "cpu_model": None, "smt": None}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        with open("/sys/devices/system/cpu/smt/active") as f:
            info["smt"] = f.read().strip() == "1"
    except OSError:
        pass
    return info


def graph_search_leg(idx, w, Q, gt, torch, bridged, seeds_count=16):
    """The neighborhood-graph search without bridges (Sec. 2.2, the iterative
    search Sec. 5.3 compares against): fixed seeds, best first over the kNN
    graph, on the same budgets as the bridged search, doubling until it too
    reaches recall@10 >= 0.9 (or 16384)."""
    from paper_1312_3062_amd import recall_at, synth
    qd = torch.from_numpy(Q).cuda()
    seeds = torch.from_numpy(synth.graph_seeds(w, seeds_count)).cuda()
    out = (torch.empty((len(Q), w.k), dtype=torch.int32, device="cuda"),
           torch.empty((len(Q), w.k), dtype=torch.int32, device="cuda"))

    def kernel_ms(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev]))

    rows, pending = [], sorted(set(b["budget"] for b in bridged))
    from paper_1312_3062_amd._abi import AnnError
    while pending:
        T = pending.pop(0)
        try:
            g_ms = kernel_ms(lambda: idx.search_graph_device(qd, w.k, T, seeds, queue_len=w.queue_len, out=out))
        except AnnError as e:  # a budget whose visited set does not fit one workgroup's LDS
            log(f"[graph] T={T}: {e}")
            break
        g_rec = recall_at(out[0].cpu().numpy(), gt, w.k)
        b_ms = kernel_ms(lambda: idx.search_device(qd, w.k, T, queue_len=w.queue_len, out=out))
        b_rec = recall_at(out[0].cpu().numpy(), gt, w.k)
        rows.append({"budget": T, "graph_recall@10": round(g_rec, 4), "graph_kernel_ms": round(g_ms, 3),
                     "bridged_recall@10": round(b_rec, 4), "bridged_kernel_ms": round(b_ms, 3)})
        log(f"[graph] T={T}: no bridges recall@10 {g_rec:.4f} ({g_ms:.3f} ms), bridged {b_rec:.4f} ({b_ms:.3f} ms)")
        if not pending and g_rec < 0.9 and T < 16384:
            pending.append(2 * T)
    first = lambda key: next((r for r in rows if r[key] >= 0.9), None)  # noqa: E731
    g9, b9 = first("graph_recall@10"), first("bridged_recall@10")
    res = {"seeds": seeds_count, "sweep": rows}
    if g9 and b9:
        res["qps_at_recall_0.9"] = {"graph": round(len(Q) / (g9["graph_kernel_ms"] * 1e-3), 1),
                                    "bridged": round(len(Q) / (b9["bridged_kernel_ms"] * 1e-3), 1),
                                    "graph_budget": g9["budget"], "bridged_budget": b9["budget"]}
    return res


def scan_overhead_leg(idx, w, X, Q, torch, visited=10_000):
    """Fig. 5 of the paper: the time to visit `visited` reference vectors by the
    search (budget = visited) against a linear scan computing the distances to
    `visited` reference vectors (the first rows of X, on matrix cores), for the
    same queries; the overhead is the difference."""
    from paper_1312_3062_amd import knn_device
    qd = torch.from_numpy(Q).cuda()
    xs = torch.from_numpy(np.ascontiguousarray(X[:visited])).cuda()
    st = torch.empty((len(Q), 12), dtype=torch.int32, device="cuda")
    idx.search_device(qd, w.k, visited, queue_len=w.queue_len, stats=st)
    torch.cuda.synchronize()
    stn = st.cpu().numpy().astype(np.float64)
    evals = float(stn[:, 0].mean())

    def kernel_ms(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev]))

    s_ms = kernel_ms(lambda: idx.search_device(qd, w.k, visited, queue_len=w.queue_len))
    l_ms = kernel_ms(lambda: knn_device(xs, qd, w.k))
    per_q = lambda ms: ms * 1e3 / len(Q)  # noqa: E731  (microseconds per query)
    log(f"[scan] visiting {visited} vectors: search {s_ms:.3f} ms, linear scan {l_ms:.3f} ms "
        f"for {len(Q)} queries (evaluations per query {evals:.0f})")
    return {"visited": visited, "queries": len(Q), "evals_per_query": round(evals, 1),
            "ref_pops_per_query": round(float(stn[:, 1].mean()), 1), "rows_per_query": round(float(stn[:, 7].mean()), 1),
            "bridge_pops_per_query": round(float(stn[:, 2].mean()), 1),
            "search_ms": round(s_ms, 3), "linear_scan_ms": round(l_ms, 3),
            "search_us_per_query": round(per_q(s_ms), 3), "linear_scan_us_per_query": round(per_q(l_ms), 3),
            "overhead_us_per_query": round(per_q(s_ms - l_ms), 3), "ratio": round(s_ms / max(l_ms, 1e-9), 2)}


def graph_d_adc_leg(X, Q, gt1, torch, lists=6144, ms=(8, 16), lengths=(10_000, 30_000, 100_000), pq_iters=4,
                    assign_budget=256, seed=7, cpu_sample=50):
    """Sec. 5 (Table 2's protocol on synthetic data): inverted lists over
    `lists` coarse centres (a seeded sample of the vectors, about 163 vectors
    a list as 1B / 6M in the paper), each vector assigned by the graph search
    over the centres, its residual product-quantised into m bytes; a query
    visits its nearest lists until L candidates and re-ranks them by the
    asymmetric distance.  The centres' index: kNN graph of 16, two subspaces
    of 16 codewords, every centre linked from its nearest bridge; the lists
    come from a search with budget 4W for W lists.  R@T: share of queries
    whose true nearest neighbour is within the first T re-ranked candidates.
    Beside each row the oracle (lists by its search over the exported
    centres' index, then its fp64 re-ranking) is timed single-threaded on the
    first `cpu_sample` queries, and its ids compared with the GPU's."""
    from paper_1312_3062_amd.ivf import Ivf
    qd = torch.from_numpy(Q).cuda()
    nq = len(Q)
    out = []
    for m in ms:
        t0 = time.time()
        ivf = Ivf.build(X, lists=lists, pq_m=m, pq_iters=pq_iters, assign_budget=assign_budget, seed=seed,
                        graph_k=16, P=2, K=16, kmeans_iters=4, bridge_t=1, bridge_b=0, centre_seed=seed)
        torch.cuda.synchronize()
        build_s = time.time() - t0
        parts = ivf.export()
        off = parts["list_off"].astype(np.int64)
        sizes = np.diff(off)
        cidx = ivf.centres_index()
        cparts = cidx.export()
        log(f"[adc] m={m}: built in {build_s:.1f}s, {lists} lists of {sizes.mean():.0f} vectors on average "
            f"(largest {sizes.max()}, empty {int((sizes == 0).sum())})")
        for L in lengths:
            W = int(min(1024, np.ceil(1.5 * L / max(1.0, sizes.mean()))))
            Tc = max(256, 4 * W)

            def ms_of(fn, reps=3):
                fn()
                torch.cuda.synchronize()
                ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                      for _ in range(reps)]
                for a, b in ev:
                    a.record()
                    fn()
                    b.record()
                torch.cuda.synchronize()
                return float(np.mean([a.elapsed_time(b) for a, b in ev]))

            res = {}
            total_ms = ms_of(lambda: res.update(r=ivf.search_device(qd, 100, W, Tc, L)))
            lists_ms = ms_of(lambda: cidx.search_device(qd, W, Tc))
            ids = res["r"][0].cpu().numpy()
            gl, _ = cidx.search_device(qd, W, Tc)
            gl = gl.cpu().numpy().astype(np.int64)
            cand = np.minimum(np.where(gl >= 0, sizes[np.maximum(gl, 0)], 0).sum(1), L)
            hit = ids == gt1[:, None]
            rec = {f"R@{t}": round(float(hit[:, :t].any(1).mean()), 4) for t in (1, 10, 100)}
            adc_ms = total_ms - lists_ms
            adc_bytes = float(cand.sum()) * (m + 4)   # code + beta per candidate
            row = {"m": m, "L": L, "lists_visited": W, "centre_budget": Tc,
                   "candidates_per_query": round(float(cand.mean()), 1), **rec,
                   "batch_ms": round(total_ms, 3), "list_search_ms": round(lists_ms, 3), "adc_ms": round(adc_ms, 3),
                   "qps": round(nq / (total_ms * 1e-3), 1), "us_per_query": round(total_ms * 1e3 / nq, 3),
                   "adc_GBps": round(adc_bytes / max(adc_ms, 1e-6) / 1e6, 1),
                   "adc_frac": round(adc_bytes / max(adc_ms, 1e-6) / 1e6 / HBM_PEAK_GBS, 4),
                   "build_s": round(build_s, 1)}
            if cpu_sample:
                import oracle
                qs = Q[:cpu_sample]
                t0 = time.perf_counter()
                olists, _ = oracle.search(parts["centres"], cparts["codebooks"], cparts["graph"], cparts["bridge_off"],
                                          cparts["bridge_ids"], qs, W, Tc, 64)
                oids, _ = oracle.ivf_adc(qs, parts["centres"], parts["list_off"], parts["list_ids"], parts["codes"],
                                         parts["pq"], olists, L, 100)
                cpu_s = time.perf_counter() - t0
                row["cpu_baseline"] = {
                    "value": round(cpu_sample / cpu_s, 1), "unit": "queries/s", "cores": 1, "kind": "oracle",
                    "sample": f"first {cpu_sample} queries ({cpu_s:.2f} s): the oracle's search for the lists, then "
                              f"its fp64 re-ranking",
                    "lists_equal": bool(np.array_equal(olists, gl[:cpu_sample])),
                    "ids_equal_share": round(float((oids == ids[:cpu_sample]).mean()), 4)}
            log(f"[adc] m={m} L={L}: lists {W}, {row['candidates_per_query']:.0f} candidates, {rec}, "
                f"{total_ms:.2f} ms per {nq} queries (lists {lists_ms:.2f}), {row['qps']:.0f} QPS"
                + (f"; oracle {row['cpu_baseline']['value']:.0f} QPS, lists equal "
                   f"{row['cpu_baseline']['lists_equal']}, ids equal {row['cpu_baseline']['ids_equal_share']}"
                   if cpu_sample else ""))
            out.append(row)
        ivf.close()
    return {"lists": lists, "n": len(X), "queries": nq, "pq_iters": pq_iters, "assign_budget": assign_budget,
            "results": out}


def oracle_all_cores(oracle, X, parts, Q, sample, passes, w, T, gpu_ids):
    """The same oracle sample spread over the host's cores: one thread per
    slice of the queries (the C oracle runs outside the interpreter lock),
    `passes` passes as in the single-threaded timing."""
    from concurrent.futures import ThreadPoolExecutor
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    bounds = np.linspace(0, sample, cores + 1).astype(int)

    def part(i):
        lo, hi = bounds[i], bounds[i + 1]
        if hi <= lo:
            return lo, np.empty((0, w.k), np.int32)
        oi, _ = oracle.search(X, parts["codebooks"], parts["graph"], parts["bridge_off"], parts["bridge_ids"],
                              Q[lo:hi], w.k, T, w.queue_len)
        return lo, oi

    same = True
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        for _ in range(passes):
            for lo, oi in ex.map(part, range(cores)):
                same = same and bool(np.array_equal(oi, gpu_ids[lo:lo + len(oi)]))
    secs = time.perf_counter() - t0
    return {"value": round(sample * passes / secs, 2), "unit": "queries/s", "cores": cores,
            "cap": "at most 16 threads: the host's CPU share for one GPU",
            "sample": f"the same {sample} queries x {passes} passes split over {cores} threads ({secs:.1f} s); "
                      f"ids identical to the GPU: {same}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sift_like_1m_u8")
    ap.add_argument("--budget", type=int, default=0,
                    help="fixed budget T (0: the smallest budget on the refined grid with recall >= target)")
    ap.add_argument("--target-recall", type=float, default=0.9)
    ap.add_argument("--cpu-sample", type=int, default=0, help="queries for the oracle baseline (0: auto)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-vs-plain request streams")
    ap.add_argument("--serve-requests", type=int, default=5000, help="requests per served / plain run")
    ap.add_argument("--serve-requests-10m", type=int, default=2000,
                    help="requests per served / plain run of the mixed stream on the 10M index")
    ap.add_argument("--serve-loads", type=float, nargs="+", default=[0.5, 1.1, 2.0, 4.0],
                    help="request rates as multiples of the plain saturation rate")
    ap.add_argument("--serve-mixed", action="store_true",
                    help="also serve a stream with k in {1,10,100} and budgets 128..8192 per request")
    ap.add_argument("--serve-pool", type=int, default=800_000, help="query vectors the request streams draw")
    ap.add_argument("--bridge-t", type=int, default=-1, help="override the workload's bridges per vector (t)")
    ap.add_argument("--bridge-b", type=int, default=-1, help="override the workload's vectors per bridge (b; 0 = all)")
    ap.add_argument("--sweep-bridges", action="store_true",
                    help="sweep the bridge rule (t, b) and the codebooks (P, K) instead of the benchmark")
    ap.add_argument("--no-scale", action="store_true",
                    help="skip the 10M x 128 legs (uneven batch, mixed request stream)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the graph search without bridges and the linear-scan overhead legs")
    ap.add_argument("--adc-only", action="store_true", help="run the Graph-D-ADC leg alone")
    ap.add_argument("--copy-probe", action="store_true",
                    help="end with a copy-like kernel over 1 GiB (calibrates hardware traffic counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the search shards by query with a replicated index, "
              "so no multi-GPU figure is produced (run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1312_3062_amd import Index, knn_device, recall_at, synth

    w = synth.WORKLOADS[args.workload]
    overridden = args.bridge_t >= 0 or args.bridge_b >= 0
    if overridden:
        import dataclasses
        w = dataclasses.replace(w, bridge_t=w.bridge_t if args.bridge_t < 0 else args.bridge_t,
                                bridge_b=w.bridge_b if args.bridge_b < 0 else args.bridge_b)
    if args.sweep_bridges:
        bridge_sweep(w, args, torch)
        return
    if w.variable_kT:
        bench_uneven(w, args, torch)
        return
    if args.adc_only:
        X, Q = synth.base_vectors(w), synth.queries(w)
        xd, qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
        gt, _ = knn_device(xd, qd, 1)
        torch.cuda.synchronize()
        del xd
        line = {"graph_d_adc": graph_d_adc_leg(X, Q, gt.cpu().numpy()[:, 0], torch)}
        if args.copy_probe:
            copy_probe(torch)
        print(json.dumps(line), flush=True)
        return
    t0 = time.time()
    X = synth.base_vectors(w)
    Q = synth.queries(w)
    log(f"[bench] data {X.shape} {X.dtype}, queries {Q.shape} in {time.time() - t0:.1f}s")
    torch.cuda.set_device(0)
    t0 = time.time()
    idx = Index.build(X, w.graph_k, w.P, w.K, w.kmeans_iters, w.kmeans_seed, w.bridge_t, w.bridge_b)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    info = idx.info
    log(f"[bench] index built in {build_s:.1f}s: {info}")
    alpha = bridge_alpha(idx)
    log(f"[bench] bridge graph: {alpha['linked']} reference vectors linked, alpha {alpha['alpha']:.4f}; "
        f"{alpha['nonempty_share']:.4f} of the K^P lists not empty")

    xd = torch.from_numpy(X).cuda()
    qd = torch.from_numpy(Q).cuda()
    t0 = time.time()
    if X.dtype == np.uint8:
        gt, _ = knn_device(xd, qd, w.k)
        torch.cuda.synchronize()
        gt = gt.cpu().numpy()
    else:
        gt = gt_f32(X, xd, Q, w.k, torch, knn_device)
    log(f"[bench] ground truth (GPU linear scan{'' if X.dtype == np.uint8 else ', fp64 re-rank'}) "
        f"in {time.time() - t0:.1f}s")
    big = None
    if X.dtype == np.float32:
        # ten times the batch, same recipe: the throughput case of the precision comparison
        bq = synth.queries(w, 10 * len(Q))
        big = (bq, gt_f32(X, xd, bq, w.k, torch, knn_device))
    del xd

    nq = Q.shape[0]
    stats = torch.empty((nq, 12), dtype=torch.int32, device="cuda")
    grid = [args.budget] if args.budget else list(w.budgets)
    sweep = []
    chosen = None
    def run(T):
        ids, dd = idx.search_device(qd, w.k, T, queue_len=w.queue_len, stats=stats)
        torch.cuda.synchronize()
        st = stats.cpu().numpy()
        if (st[:, 6] != 0).any():
            raise RuntimeError(f"T={T}: {int((st[:, 6] != 0).sum())} queries overflowed a per-query structure")
        rec = recall_at(ids.cpu().numpy(), gt, w.k)
        sweep.append({"budget": T, "recall@10": round(rec, 4)})
        log(f"[bench] T={T} recall@{w.k}={rec:.4f} evals={st[:, 0].mean():.0f} ref_pops={st[:, 1].mean():.0f} "
            f"bridge_pops={st[:, 2].mean():.0f} bridges_gen={st[:, 4].mean():.0f} heap_max={st[:, 5].max()} "
            f"rows={st[:, 7].mean():.0f} lookaheads={st[:, 8].mean():.0f}")
        return T, rec, st

    # doubling grid first, then the smallest budget reaching the target
    # between the last two grid points, in steps of an eighth of the lower one
    prev = None
    for T in grid:
        chosen = run(T)
        if chosen[1] >= args.target_recall:
            break
        prev = T
    if not args.budget and prev is not None and chosen[1] >= args.target_recall:
        step = max(16, prev // 8)
        for T in range(prev + step, chosen[0], step):
            c = run(T)
            if c[1] >= args.target_recall:
                chosen = c
                break
    T, rec, st = chosen

    # timed region: K whole-batch searches, HIP events on the launch stream
    stream = torch.cuda.current_stream()
    out = (torch.empty((nq, w.k), dtype=torch.int32, device="cuda"),
           torch.empty((nq, w.k), dtype=torch.int32 if X.dtype == np.uint8 else torch.float32, device="cuda"))

    def timed(tune):
        for _ in range(args.warmup):
            idx.search_device(qd, w.k, T, queue_len=w.queue_len, out=out, tune=tune)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        t_wall = time.perf_counter()
        for a, b in ev:
            a.record(stream)
            idx.search_device(qd, w.k, T, queue_len=w.queue_len, out=out, tune=tune)
            b.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_wall
        return wall, float(np.mean([a.elapsed_time(b) for a, b in ev]))

    plain_wall, plain_kms = timed(None)
    log(f"[bench] plain launch: {plain_kms:.3f} ms kernel, {nq * args.steps / plain_wall:.0f} QPS")
    tune = idx.autotune(qd, w.k, T, queue_len=w.queue_len)
    log(f"[bench] autotuned launch setting: {tune}")
    wall, kms = timed(tune)
    ms_step = wall * 1000.0 / args.steps
    qps = nq * args.steps / wall
    log(f"[bench] tuned launch: {kms:.3f} ms kernel, {qps:.0f} QPS")

    # the same batch through the host-buffer entry point: queries copied in,
    # results copied out, device buffers set up per call (reported beside the
    # device-resident value, never as it)
    idx.search(Q, w.k, T, queue_len=w.queue_len)
    t_host = time.perf_counter()
    host_reps = 3
    for _ in range(host_reps):
        idx.search(Q, w.k, T, queue_len=w.queue_len)
    host_qps = nq * host_reps / (time.perf_counter() - t_host)
    log(f"[bench] host buffers (copies in and out included): {host_qps:.0f} QPS")

    d_bytes = X.shape[1] * X.itemsize
    B = algorithmic_bytes(st, d_bytes, w.graph_k, w.k, d_bytes)
    achieved = float(B.sum()) / (kms * 1e-3) / 1e9
    log(f"[bench] T={T}: {ms_step:.3f} ms/step wall, kernel {kms:.3f} ms, QPS {qps:.0f}, "
        f"algorithmic {B.sum() / 1e9:.3f} GB/launch -> {achieved:.1f} GB/s")

    if args.copy_probe:
        copy_probe(torch)

    # HBM traffic of the search kernel, from the counter runs kept with the
    # profiles (only if taken on the current kernel sources and this workload)
    from paper_1312_3062_amd.profiling import read_traffic_record
    trec = read_traffic_record(os.path.join(ROOT, "profiles", f"k_search_{w.name}_traffic.md"))
    traffic = (trec["bytes_per_launch"] if trec and trec.get("workload") == f"{w.name} T={T} nq={nq}" and not overridden
               else None)

    precision = None
    if X.dtype == np.float32:
        precision = precision_leg(idx, w, X, Q, gt, T, torch, big=big)
        log(f"[bench] precision: {precision}")

    serving = None
    if not args.no_serve and X.dtype == np.uint8:
        xd2 = torch.from_numpy(X).cuda()

        def gt_fn(qs):
            ids_, _ = knn_device(xd2, torch.from_numpy(np.ascontiguousarray(qs)).cuda(), 10)
            torch.cuda.synchronize()
            return ids_.cpu().numpy()

        serving = {"operating_point": serving_leg(idx, w, args, gt_fn, fixed_k=w.k, fixed_budget=T)}
        if args.serve_mixed:
            serving["mixed_k_budget"] = serving_leg(idx, w, args, gt_fn)
        del xd2

    graph_leg = scan_leg = adc_leg = None
    if not args.no_extra and X.dtype == np.uint8:
        graph_leg = [graph_search_leg(idx, w, Q, gt, torch, sweep, seeds_count=c) for c in (16, 256)]
        scan_leg = scan_overhead_leg(idx, w, X, Q, torch)
        try:
            adc_leg = graph_d_adc_leg(X, Q, gt[:, 0], torch)
        except Exception as e:  # reported in the line; the headline above stands
            log(f"[bench] Graph-D-ADC leg failed: {e!r}")
            adc_leg = {"error": repr(e)}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        parts = idx.export()
        # about 10 s of single-threaded work: the first `sample` queries, passes
        # over them repeated until 10 s have gone by (at most 4 passes)
        sample = args.cpu_sample or max(20, min(nq, int(40000 * 1024 / max(T, 1))))
        passes, cpu_s, same = 0, 0.0, True
        while passes < 4 and (passes == 0 or cpu_s < 10.0):
            t0 = time.perf_counter()
            oi, _ = oracle.search(X, parts["codebooks"], parts["graph"], parts["bridge_off"], parts["bridge_ids"],
                                  Q[:sample], w.k, T, w.queue_len)
            cpu_s += time.perf_counter() - t0
            passes += 1
            same = same and bool(np.array_equal(oi, out[0][:sample].cpu().numpy()))
        done = sample * passes
        cpu = {"value": round(done / cpu_s, 2), "unit": "queries/s", "cores": 1, "kind": "oracle",
               "sample": f"first {sample} of {nq} queries x {passes} passes at T={T} ({cpu_s:.1f} s), "
                         f"single-threaded C oracle on the GPU-built index; ids identical to the GPU: {same}",
               "host": host_info()}
        log(f"[bench] oracle: {done} queries in {cpu_s:.1f}s -> {done / cpu_s:.1f} QPS (ids equal: {same})")
        cpu["all_cores"] = oracle_all_cores(oracle, X, parts, Q, sample, passes, w, T, out[0][:sample].cpu().numpy())
        log(f"[bench] oracle on {cpu['all_cores']['cores']} threads: {cpu['all_cores']['value']} QPS")

    if X.dtype == np.uint8:
        metric = f"QPS at recall@10>={args.target_recall:g}, {w.n // 1_000_000}M x{w.d} uint8"
    else:
        metric = f"QPS at budget {T}, {w.n // 1_000_000}M x{w.d} fp32"
    line = {
        "metric": metric,
        "value": round(qps, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8" if X.dtype == np.uint8 else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "d": w.d, "queries": nq, "k": w.k, "budget": T,
                   "queue_len": w.queue_len, "graph_k": w.graph_k, "P": w.P, "K": w.K,
                   "bridge_t": w.bridge_t, "bridge_b": w.bridge_b, "recall@10": round(rec, 4),
                   "budget_sweep": sweep, "launch": tune, "build_s": round(build_s, 2),
                   "plain_qps": round(nq * args.steps / plain_wall, 1), "plain_kernel_ms": round(plain_kms, 4),
                   "host_buffers_qps": round(host_qps, 1),
                   "bridge_alpha": round(alpha["alpha"], 5), "bridges_nonempty": round(alpha["nonempty_share"], 5)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "kernel": "k_search", "kernel_ms": round(kms, 4),
                     "algorithmic_bytes_per_launch": int(B.sum())},
        "cpu_baseline": cpu,
        "serving": serving,
        "precision": precision,
        "graph_search_without_bridges": graph_leg,
        "overhead_vs_linear_scan": scan_leg,
        "graph_d_adc": adc_leg,
    }
    if not args.no_scale and X.dtype == np.uint8 and not overridden:
        # the 10M x 128 workload: its uneven batch (a second roofline figure,
        # the HBM-resident case) and the mixed request stream served over it
        del idx, qd, out, stats
        torch.cuda.empty_cache()
        try:
            line["scale_10m"] = uneven_leg(synth.WORKLOADS["hog_like_10m_u8"], args, torch,
                                           serve_mixed=not args.no_serve, cpu_baseline=False)
        except Exception as e:  # reported in the line; the headline above stands
            log(f"[bench] 10M leg failed: {e!r}")
            line["scale_10m"] = {"error": repr(e)}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
