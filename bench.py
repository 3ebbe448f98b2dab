"""t-SGNE throughput benchmark on one MI355X.

One step = one pass of the whole hot path over one graph: affinities
(tsgne_build_P), n_iter optimisation steps (tsgne_run: repulsion + Z,
attraction, update) and the final KL (tsgne_kl).  Inputs are synthetic and
already resident in HBM when the timed region starts.  The default workload
is the 300,000-node / 1,000,000-edge DC-SBM with 128-dim embeddings and 1000
iterations.

value = pair interactions per second over the whole job
      = steps * n_iter * n(n-1) / elapsed.

Prints one JSON line (rank 0).  Also reports the roofline of the dominant
kernel (the repulsion, timed with HIP events on its own stream; the layouts
of the timed region run with phase timing on, so each step's launches are
issued one by one between events; for layouts under 2 s, the time of a
layout without phase timing, whose steps replay captured chunks, is reported
beside it as layout_ms_replayed), the FP64 oracle timed on the host cores
over a bounded sample, and, for the default workload, a compact serving leg
(48 requests of 1K-200K nodes, 500 iterations each: saturated and Poisson
arrivals at 0.8x the saturated rate, continuous batching against one request
at a time).
"""
from __future__ import annotations

import argparse
import hashlib
import math
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published FP32 vector peak (packed FMA)
FLOP_PER_PAIR = 13                # algorithmic flops per ordered pair of the repulsion
FP32_NONPACKED_FMA_TFLOPS = 78.6  # 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz (packed FP32 disabled)
# FP32 flop the hardware counts per unordered pair in the symmetric repulsion
# (rocprofv3 SQ_INSTS_VALU_FLOPS_FP32 x 64 lanes / unordered pairs, FMA = 2;
# 15 rows per lane, the 300K tile; 17.17 with 14 rows)
EXECUTED_FLOP_PER_UNORDERED_PAIR = 17.165
PROFILE_DIR = os.path.join(ROOT, "profiles")


def log(msg: str) -> None:
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("step.hip", "internal.h"):
        with open(os.path.join(ROOT, "paper_2310_11186_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def repulse_kernel_name(rows: int, split: bool = True, symmetric: bool = True) -> str:
    """The repulsion kernel instantiation a run launches, as the profiler names it."""
    return "k_repulse<%d, %s, %s>" % (rows, "true" if split else "false", "true" if symmetric else "false")


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per repulsion launch from the committed counter summary, if it
    was taken on the current kernel source and on the same kernel
    instantiation (tile size, precision, variant) as this run; else None."""
    path = os.path.join(PROFILE_DIR, "repulsion_%s_traffic.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_hash") != kernel_source_hash() or rec.get("kernel") != kernel:
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(gi, n_iter_total: int, exaggeration_iters: int, perplexity: float, budget_s: float):
    """FP64 oracle on the host: optimisation steps on a 20,000-node snowball
    sample of the same graph, timed until ~budget_s seconds have passed."""
    import numpy as np

    import oracle
    from paper_2310_11186_amd import synth
    sub = synth.snowball_sample(gi, 20_000, seed=1)
    size, e = sub.n, sub.edges
    rp, col = oracle.csr_from_edges(size, e)
    P, _ = oracle.build_P(rp, col, sub.X, perplexity)
    Y = sub.Y0.astype(np.float64)
    U = np.zeros_like(Y)
    G = np.ones_like(Y)
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and steps < n_iter_total:
        Y, U, G, _ = oracle.run(rp, col, P, Y, U, G, t0=steps, n_steps=1, exaggeration_iters=exaggeration_iters,
                                eta=max(size / 48.0, 50.0))
        steps += 1
    dt = time.perf_counter() - t0
    pairs = steps * size * (size - 1)
    return {
        "value": pairs / dt,
        "unit": "pair-interactions/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": "%d full FP64 oracle steps (all-pairs gradient + update) on a %d-node, %d-edge BFS snowball "
                  "sample of the same graph, %.1f s" % (steps, size, e.shape[0], dt),
    }


def run_batch(args) -> int:
    """256 independent SBM graphs, 750 iterations each: batched (one captured
    step replayed, tile chosen by the autotuner) against one graph at a time
    (tsgne_run with each graph's default plan), on the same GPU."""
    import numpy as np
    import torch

    from paper_2310_11186_amd import synth, tsgne

    dev = torch.device("cuda:0")
    n_iter = args.n_iter if args.n_iter is not None else 750
    t_ee = n_iter // 4
    log("generating 256 SBM graphs")
    gis = synth.batch_workload()
    graphs, X0 = [], []
    t0 = time.perf_counter()
    for gi in gis:
        rp, col = tsgne.tsgne_csr_from_edges(gi.n, gi.edges)
        graphs.append(tsgne.tsgne_build_P(torch.from_numpy(rp).to(dev), torch.from_numpy(col).to(dev),
                                          torch.from_numpy(gi.X).to(dev), 30.0))
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    Y0 = [torch.from_numpy(gi.Y0).to(dev) for gi in gis]
    params = tsgne.tsgne_params_default(exaggeration_iters=t_ee)
    best, ms = tsgne.tsgne_autotune(graphs, Y0, params, steps=3)
    log("autotuner (one tile): ms/step for tile_rows %s = %s -> %d" %
        (tsgne.AUTOTUNE_TILES, ["%.2f" % m for m in ms], best))
    t_tune = time.perf_counter()
    tiles, ms_uniform, ms_tuned = tsgne.tsgne_autotune_tiles(graphs, Y0, params, steps=3)
    tune_s = time.perf_counter() - t_tune
    by_bucket = {}
    for gi, t in zip(gis, tiles):
        by_bucket[int(math.floor(math.log2(gi.n)))] = t
    log("autotuner (tile per size bucket, %.1f s): %s, %.2f -> %.2f ms/step" %
        (tune_s, by_bucket, ms_uniform, ms_tuned))
    params_b = tsgne.tsgne_params_default(exaggeration_iters=t_ee, repulsion=tsgne.TSGNE_REPULSION_SYMMETRIC)
    params_u = tsgne.tsgne_params_default(exaggeration_iters=t_ee, tile_rows=best)
    pairs = sum(float(gi.n) * (gi.n - 1) for gi in gis) * n_iter

    def padded_pairs(rows_of):
        tot = 0.0
        for gi, R in zip(gis, rows_of):
            T = 64 * R
            nb = (gi.n + T - 1) // T
            tot += float(nb * T) ** 2
        return tot

    padding = {"tuned": padded_pairs(tiles) / (pairs / n_iter) - 1.0,
               "one_tile": padded_pairs([best] * len(gis)) / (pairs / n_iter) - 1.0}

    Yb = [y.clone() for y in Y0]
    tsgne.tsgne_batch_run_tiles(graphs[:8], Yb[:8], [5] * 8, tiles[:8], params_b)   # warm-up of the batched path
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        Yb = [y.clone() for y in Y0]
        tsgne.tsgne_batch_run_tiles(graphs, Yb, [n_iter] * len(graphs), tiles, params_b)
    torch.cuda.synchronize()
    batched_s = (time.perf_counter() - t0) / args.steps
    log("batched, tuned tiles: %.2f s per 256 layouts" % batched_s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Yb = [y.clone() for y in Y0]
    tsgne.tsgne_batch_run(graphs, Yb, [n_iter] * len(graphs), params_u)
    torch.cuda.synchronize()
    uniform_s = time.perf_counter() - t0
    log("batched, one tile (%d): %.2f s" % (best, uniform_s))

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Ys = [y.clone() for y in Y0]
    for g, y in zip(graphs, Ys):
        tsgne.tsgne_run(g, y, n_iter, params)
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t0
    log("one at a time: %.2f s" % seq_s)
    result = {
        "metric": "batched t-SGNE pair-interactions/s (256 SBM graphs, 750 iterations each)",
        "value": pairs / batched_s,
        "unit": "pair-interactions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": batched_s * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 (FP64 Z/KL/cross-tile sums)",
        "data": "synthetic",
        "config": {"workload": "batch256", "graphs": len(gis), "nodes_total": int(sum(gi.n for gi in gis)),
                   "sum_n2": float(sum(float(gi.n) ** 2 for gi in gis)), "n_iter": n_iter, "d": 64,
                   "tile_rows_by_size_bucket": by_bucket, "autotune_s": tune_s,
                   "autotune_ms_per_step": {"one_tile": ms_uniform, "tuned": ms_tuned},
                   "padding_of_pair_work": padding, "build_P_s": build_s},
        "layouts_per_s": len(gis) / batched_s,
        "one_tile": {"tile_rows": best, "seconds": uniform_s, "autotune_ms_per_step": ms,
                     "pair_interactions_per_s": pairs / uniform_s},
        "one_at_a_time": {"seconds": seq_s, "pair_interactions_per_s": pairs / seq_s,
                          "layouts_per_s": len(gis) / seq_s},
        "speedup_vs_one_at_a_time": seq_s / batched_s,
    }
    print(json.dumps(result), flush=True)
    for g in graphs:
        g.close()
    return 0


def request_pool(workers: int = 16):
    """Worker processes that generate serving requests ahead of their arrival.
    Made by fork before this process touches the GPU: the workers only run
    numpy generators."""
    import multiprocessing as mp
    return mp.get_context("fork").Pool(processes=max(1, min(workers, os.cpu_count() or 1)))


def serve_stream(srv_kwargs, specs, arrivals, n_iter, pool=None, reqs=None, label="stream"):
    """Submits the requests of `specs` (or the generated `reqs`) at the given
    arrival times (s) and waits for all; returns the server's statistics (with
    each request's (latency ms, queued ms) in submission order) and the wall
    time.  With a pool, each request is generated by the pool ahead of its
    arrival and dropped once the server has copied it in."""
    from paper_2310_11186_amd import synth, tsgne
    feed = iter(reqs) if reqs is not None else pool.imap(synth.serving_request, specs, chunksize=1)
    srv = tsgne.Server(**srv_kwargs)
    t0 = time.perf_counter()
    tickets = []
    count = len(specs)
    for k, at in enumerate(arrivals):
        gi = next(feed)
        delay = at - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.submit(gi.n, gi.edges, gi.X, gi.Y0, 30.0, n_iter))
        del gi
        if count >= 200 and (k + 1) % 100 == 0:
            st = srv.stats()
            log("%s: %d/%d submitted, %d completed, %.0f s" % (label, k + 1, count, st["completed"],
                                                                  time.perf_counter() - t0))
    statuses = [srv.wait(t)[0] for t in tickets]
    wall = time.perf_counter() - t0
    st = srv.stats()
    times = [srv.latency(t) for t in tickets]
    srv.close()
    if any(s != tsgne.TSGNE_OK for s in statuses):
        raise RuntimeError("a served request failed: %s" % statuses)
    st["per_request"] = times
    return st, wall


def nearest_rank(values, q):
    """The q-quantile by nearest rank (the server's own definition)."""
    v = sorted(values)
    return v[min(len(v), max(1, math.ceil(q * len(v)))) - 1] if v else None


def by_size_decile(sizes, st):
    """p50 / max latency (ms) of the requests in each tenth of the node counts."""
    order = sorted(range(len(sizes)), key=lambda k: sizes[k])
    out = []
    for d in range(10):
        idx = order[d * len(order) // 10:(d + 1) * len(order) // 10]
        if not idx:
            continue
        lat = [st["per_request"][k][0] for k in idx]
        out.append({"decile": d + 1, "nodes": [sizes[idx[0]], sizes[idx[-1]]], "requests": len(idx),
                    "latency_p50_ms": nearest_rank(lat, 0.5), "latency_max_ms": max(lat)})
    return out


def slowest(st, sizes, arrivals, top=3):
    """The `top` slowest requests: submission index, nodes, arrival (s),
    latency and wait for admission (ms)."""
    lat = st["per_request"]
    order = sorted(range(len(lat)), key=lambda k: -lat[k][0])[:top]
    return [{"request": k, "nodes": int(sizes[k]), "arrival_s": round(float(arrivals[k]), 3),
             "latency_ms": lat[k][0], "queued_ms": lat[k][1]} for k in order]


def stream_summary(st, wall, count):
    return {"layouts_per_s": count / wall, "latency_p50_ms": st["latency_p50_ms"],
            "latency_p99_ms": st["latency_p99_ms"], "latency_mean_ms": st["latency_mean_ms"],
            "queued_max_ms": max(q for _, q in st["per_request"]), "seconds": wall,
            "worker_s": {"rounds": st["busy_s"], "admission": st["admit_s"], "planning": st["plan_s"]},
            "rounds": st["rounds"]}


def poisson_arrivals(count, qps, seed=2310_11186):
    import numpy as np
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / qps, size=count))


def serve_kwargs(n_iter, tile_rows=0, round_ms=25.0):
    from paper_2310_11186_amd import tsgne
    params = tsgne.tsgne_params_default(exaggeration_iters=n_iter // 4)
    return dict(max_active=64, steps_per_round=512, round_ms=round_ms, tile_rows=tile_rows, params=params)


def serving_leg(reqs, n_iter):
    """The compact serving measurement of the default line: the stream all at
    once (saturated) and Poisson arrivals at 0.8x the saturated rate, each
    with continuous batching (the server's default policy) and one request at
    a time."""
    specs = [None] * len(reqs)
    count = len(reqs)
    sizes = [g.n for g in reqs]
    kw = serve_kwargs(n_iter)
    kw1 = dict(kw, max_active=1)
    st_sat, wall_sat = serve_stream(kw, specs, [0.0] * count, n_iter, reqs=reqs)
    st_sat1, wall_sat1 = serve_stream(kw1, specs, [0.0] * count, n_iter, reqs=reqs)
    sat_rate = count / wall_sat
    log("serving leg, saturated: %.2f layouts/s batched, %.2f one at a time" % (sat_rate, count / wall_sat1))
    arrivals = poisson_arrivals(count, 0.8 * sat_rate)
    st, wall = serve_stream(kw, specs, arrivals, n_iter, reqs=reqs)
    st1, wall1 = serve_stream(kw1, specs, arrivals, n_iter, reqs=reqs)
    log("serving leg, 0.8x: p50 %.0f / p99 %.0f ms batched, %.0f / %.0f one at a time" %
        (st["latency_p50_ms"], st["latency_p99_ms"], st1["latency_p50_ms"], st1["latency_p99_ms"]))
    return {
        "metric": "served layouts/s and p50/p99 latency (Poisson arrivals at 0.8x the saturated rate)",
        "requests": count, "n_iter": n_iter, "nodes_range": [min(g.n for g in reqs), max(g.n for g in reqs)],
        "policy": "short-first: short requests first, long ones one at a time in submission order",
        "saturated_layouts_per_s": sat_rate, "saturated_one_at_a_time_layouts_per_s": count / wall_sat1,
        "saturated_speedup": wall_sat1 / wall_sat, "qps": 0.8 * sat_rate,
        "batched": dict(stream_summary(st, wall, count), slowest=slowest(st, sizes, arrivals)),
        "one_at_a_time": dict(stream_summary(st1, wall1, count), slowest=slowest(st1, sizes, arrivals)),
        "note": "served figures include host-to-device copies of each request and the copy of each layout back",
    }


def run_serve(args) -> int:
    """Serving: layout requests with Poisson arrivals at fractions of the
    measured saturated rate (0.8 is the headline), continuous batching (the
    default short-first policy, and the earlier oldest-share policy) against
    one request at a time, latency by request size, and a run under a small
    device-memory budget that makes requests queue for memory.  Long streams
    (--requests in the thousands) are generated by worker processes ahead of
    their arrival; --serve-qps fixes the arrival rate (no saturated runs) and
    --serve-only runs a single configuration."""
    from paper_2310_11186_amd import synth, tsgne

    pool = request_pool()
    count = args.requests
    n_iter = args.n_iter if args.n_iter is not None else 500
    specs = synth.serving_request_specs(count)
    sizes = [sp[1] for sp in specs]
    kw = serve_kwargs(n_iter, args.tile_rows, args.serve_round_ms)
    kw1 = dict(kw, max_active=1)
    kw_old = dict(kw, rest_policy=tsgne.TSGNE_SHARE_EQUAL, oldest_share=0.5)
    configs = {"batched": kw, "one_at_a_time": kw1, "oldest_share": kw_old}
    result = {
        "metric": "served layouts/s with p50/p99 latency (Poisson arrivals, continuous batching)",
        "unit": "layouts/s", "n_gpus": 1, "steps": 1, "warmup": 0, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (FP64 Z/KL/cross-tile sums)", "data": "synthetic",
        "config": {"workload": "serve", "requests": count, "n_iter": n_iter,
                   "nodes_range": [min(sizes), max(sizes)], "nodes_total": int(sum(sizes)),
                   "tile_rows": kw["tile_rows"], "steps_per_round": kw["steps_per_round"],
                   "round_ms": kw["round_ms"], "max_active": kw["max_active"],
                   "policy": "short-first (library default): long_ms 150, short_share 0.3"},
    }
    pairs = sum(float(n) * (n - 1) for n in sizes) * n_iter
    if args.serve_qps:
        qps = args.serve_qps
        sat_rate = qps / 0.8
    else:
        st_sat, wall_sat = serve_stream(kw, specs, [0.0] * count, n_iter, pool, label="saturated")
        sat_rate = count / wall_sat
        log("saturated: %.2f layouts/s" % sat_rate)
        result["saturated"] = {"layouts_per_s": sat_rate, "seconds": wall_sat,
                               "batched": stream_summary(st_sat, wall_sat, count)}
        if not args.serve_only:
            st_sat1, wall_sat1 = serve_stream(kw1, specs, [0.0] * count, n_iter, pool, label="saturated, one")
            log("saturated, one at a time: %.2f layouts/s" % (count / wall_sat1))
            result["saturated"].update(one_at_a_time_layouts_per_s=count / wall_sat1,
                                       speedup_vs_one_at_a_time=wall_sat1 / wall_sat,
                                       one_at_a_time=stream_summary(st_sat1, wall_sat1, count))
        if args.serve_saturated_only:
            pool.close()
            print(json.dumps(result), flush=True)
            return 0
        qps = 0.8 * sat_rate
    arrivals = poisson_arrivals(count, qps)
    result["config"]["qps"] = qps
    runs = [args.serve_only] if args.serve_only else ["batched", "one_at_a_time", "oldest_share"]
    for name in runs:
        st, wall = serve_stream(configs[name], specs, arrivals, n_iter, pool, label=name)
        log("%s at %.2f req/s: p50 %.0f ms, p99 %.0f ms, %.2f layouts/s" %
            (name, qps, st["latency_p50_ms"], st["latency_p99_ms"], count / wall))
        result[name] = dict(stream_summary(st, wall, count), by_size_decile=by_size_decile(sizes, st),
                            slowest=slowest(st, sizes, arrivals))
        if name == runs[0]:
            result["value"] = count / wall
            result["ms_per_step"] = wall * 1e3
            result["latency_p50_ms"] = st["latency_p50_ms"]
            result["latency_p99_ms"] = st["latency_p99_ms"]
            result["pair_interactions_per_s"] = pairs / wall
    if not args.serve_only and not args.serve_qps:
        load = []
        for frac in [float(v) for v in args.qps_fractions.split(",") if v]:
            if frac == 0.8:
                continue
            st_f, wall_f = serve_stream(kw, specs, poisson_arrivals(count, frac * sat_rate), n_iter, pool,
                                        label="load %.2f" % frac)
            load.append(dict(stream_summary(st_f, wall_f, count), fraction_of_saturated=frac, qps=frac * sat_rate))
            log("load %.2f x saturated: p50 %.0f ms, p99 %.0f ms" % (frac, st_f["latency_p50_ms"],
                                                                     st_f["latency_p99_ms"]))
        result["by_load"] = load
        if args.serve_low_budget_mb:
            st_lb, wall_lb = serve_stream(dict(kw, hbm_budget=args.serve_low_budget_mb << 20), specs, arrivals,
                                          n_iter, pool, label="low budget")
            result["low_budget"] = dict(stream_summary(st_lb, wall_lb, count), hbm_budget_mb=args.serve_low_budget_mb)
            log("budget %d MiB: p50 %.0f ms, p99 %.0f ms" % (args.serve_low_budget_mb, st_lb["latency_p50_ms"],
                                                             st_lb["latency_p99_ms"]))
    pool.close()
    print(json.dumps(result), flush=True)
    return 0


def run_sparse(args) -> int:
    """HBM microbenchmark of the sparse phase: the attraction kernels on a
    10M-node SBM (average degree 10, ~100M stored entries), once with the
    generator's random node numbering and once renumbered by the locality
    order of the embedding (tsgne_locality_order + tsgne_permute_graph)."""
    import torch

    from paper_2310_11186_amd import synth, tsgne

    dev = torch.device("cuda:0")
    n = args.sparse_nodes
    log("generating SBM with %d nodes" % n)
    edges, labels = synth.sbm_sparse(n, 100, 10.0, 0.18, synth.MASTER_SEED + 6)
    X = synth.embedding(labels, 8, 0.5, synth.MASTER_SEED + 6)
    Y0 = synth.initial_layout(n, synth.MASTER_SEED + 6) * 1000.0
    rp, col = tsgne.tsgne_csr_from_edges(n, edges)
    nnz = col.shape[0]
    d_rp, d_col = torch.from_numpy(rp).to(dev), torch.from_numpy(col).to(dev)
    d_X, d_Y = torch.from_numpy(X).to(dev), torch.from_numpy(Y0).to(dev)
    alg_bytes = 4 * (n + 1) + 8 * nnz + 8 * n + 16 * n

    def time_attraction(row_ptr, cols, Xn, Yn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = tsgne.tsgne_build_P(row_ptr, cols, Xn, 30.0)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        A = torch.empty((n, 2), dtype=torch.float64, device=dev)
        for _ in range(3):
            tsgne.tsgne_attraction(g, Yn, tsgne.TSGNE_PREC_SPLIT, A)
        g.set_timing(True)
        for _ in range(20):
            tsgne.tsgne_attraction(g, Yn, tsgne.TSGNE_PREC_SPLIT, A)
        ms, launches = g.timing()["attract"]
        g.close()
        return ms / launches / 1e3, build_s

    random_s, build_random_s = time_attraction(d_rp, d_col, d_X, d_Y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    perm = tsgne.tsgne_locality_order(d_X)
    o_rp, o_col = tsgne.tsgne_permute_graph(d_rp, d_col, perm)
    o_X, o_Y = tsgne.tsgne_permute_rows(d_X, perm), tsgne.tsgne_permute_rows(d_Y, perm)
    torch.cuda.synchronize()
    reorder_s = time.perf_counter() - t0
    ordered_s, build_ordered_s = time_attraction(o_rp, o_col, o_X, o_Y)
    gbs = alg_bytes / ordered_s / 1e9
    result = {
        "metric": "attraction kernel algorithmic HBM GB/s (sparse phase microbenchmark)",
        "value": gbs, "unit": "GB/s", "n_gpus": 1, "steps": 20, "warmup": 3,
        "ms_per_step": ordered_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (FP64 row sums)", "data": "synthetic",
        "config": {"workload": "sparse", "nodes": n, "stored_entries": int(nnz), "algorithmic_bytes": alg_bytes,
                   "numbering": "locality order of the embedding (Morton, 8 coordinates)",
                   "reorder_s": reorder_s, "build_P_s": build_ordered_s,
                   "random_numbering": {"ms": random_s * 1e3, "GB/s": alg_bytes / random_s / 1e9,
                                        "build_P_s": build_random_s}},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
                     "frac": gbs / 8000.0, "traffic": None},
    }
    print(json.dumps(result), flush=True)
    return 0


AQ_GRID, AQ_P = 20, 0.5


def layout_quality(Y, gi, dev, stream):
    """NMI (section 2.5) of the final layout's k-means clusters against the planted
    communities, with k = the number of communities, and AQ (section 2.6) of the
    layout coloured by the communities; computed after the timed region."""
    import numpy as np
    import torch

    from paper_2310_11186_amd import synth, tsgne

    comm = int(gi.labels.max()) + 1
    seeds = np.random.default_rng(synth.MASTER_SEED + 11).choice(gi.n, comm, replace=False).astype(np.int32)
    truth = torch.from_numpy(gi.labels.astype(np.int32)).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    labels, passes = tsgne.tsgne_kmeans(Y, torch.from_numpy(seeds).to(dev), 300, stream)
    nmi = tsgne.tsgne_nmi(truth, comm, labels, comm, stream)
    aq = tsgne.tsgne_aq(Y, truth, comm, AQ_GRID, AQ_P, stream)
    seconds = time.perf_counter() - t0
    return {"nmi": nmi, "aq": aq, "clusters": comm, "kmeans_passes": passes, "aq_grid": AQ_GRID, "aq_p": AQ_P,
            "labels": "planted communities", "seconds": seconds}


def run_sp(args) -> int:
    """The ShortestPath embedding (section 2.3, eq. (8)) of the 300,000-node,
    1,000,000-edge graph with 128 seeded random targets and l0 = sqrt(|E|)."""
    import numpy as np
    import torch

    from paper_2310_11186_amd import synth, tsgne

    dev = torch.device("cuda:0")
    gi = synth.make("dcsbm300k")
    n, d = gi.n, 128
    rp, col = tsgne.tsgne_csr_from_edges(n, gi.edges)
    nnz = col.shape[0]
    targets = np.random.default_rng(synth.MASTER_SEED + 8).choice(n, d, replace=False).astype(np.int32)
    d_rp, d_col = torch.from_numpy(rp).to(dev), torch.from_numpy(col).to(dev)
    d_t = torch.from_numpy(targets).to(dev)
    for _ in range(max(args.warmup, 1)):
        X, launched = tsgne.tsgne_shortest_path_embedding(d_rp, d_col, d_t)
    reps = max(args.steps, 5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        X, launched = tsgne.tsgne_shortest_path_embedding(d_rp, d_col, d_t)
    torch.cuda.synchronize()
    avg_s = (time.perf_counter() - t0) / reps
    l0 = float(np.sqrt(nnz // 2))
    Xh = X.cpu().numpy()
    finite = Xh[Xh <= l0]
    levels = min(int(finite.max()) + 1, int(np.floor(l0)))   # the last one finds nothing new
    W = 4
    per_level = 4 * (n + 1) + 4 * nnz + 3 * 4 * W * n      # CSR, frontier (each node's words once), vis, next frontier
    alg_bytes = levels * per_level + 4 * n * d
    result = {
        "metric": "ShortestPath embedding node-target distances/s",
        "value": n * d / avg_s, "unit": "distances/s", "n_gpus": 1, "steps": reps, "warmup": max(args.warmup, 1),
        "ms_per_step": avg_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32 bitsets, f32 output", "data": "synthetic",
        "config": {"workload": "sp_dcsbm300k", "nodes": n, "stored_entries": int(nnz), "targets": d, "l0": l0,
                   "levels_with_work": levels, "levels_launched": launched, "algorithmic_bytes": alg_bytes},
        "roofline": {"bound": "hbm", "achieved": alg_bytes / avg_s / 1e9, "peak": 8000.0, "unit": "GB/s",
                     "frac": alg_bytes / avg_s / 8e12, "traffic": None},
    }
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        oracle.shortest_path_embedding(rp, col, targets, l0)
        cpu_s = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": n * d / cpu_s, "unit": "distances/s", "cores": 1, "kind": "oracle",
                                  "sample": "the whole embedding (%d BFS), %.2f s" % (d, cpu_s)}
    print(json.dumps(result), flush=True)
    return 0


def run_shard(args) -> int:
    """One GPU's share of the repulsion of a 300,000-node layout split over
    --shards GPUs (the graph size of the default workload): each shard's call
    (tile kernel, Z reduction, per-row FP64 sums) timed in turn on this GPU.
    The value is shard 0's rate; every shard's tile-kernel time is reported to
    show the balance."""
    import numpy as np
    import torch

    from paper_2310_11186_amd import synth, tsgne

    dev = torch.device("cuda:0")
    n, G = 300_000, args.shards
    Y = torch.from_numpy(synth.initial_layout(n, synth.MASTER_SEED + 9, std=10.0)).to(dev)
    F = torch.empty((n, 2), dtype=torch.float64, device=dev)
    Z = torch.empty(1, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    reps = max(args.steps, 10)
    per_shard = []
    avg0 = None
    for s in range(G):
        sh = tsgne.Shard(n, s, G, args.tile_rows)
        R, tiles, pairs = sh.info()
        # enough warm-up calls for the clocks to settle before the first shard is timed
        for _ in range(max(args.warmup, 10)):
            sh.repulsion(Y, F=F, Z=Z, stream=stream)
        sh.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            sh.repulsion(Y, F=F, Z=Z, stream=stream)
        torch.cuda.synchronize()
        call_s = (time.perf_counter() - t0) / reps
        ms, launches = sh.timing()
        sh.close()
        tile_s = ms / launches / 1e3
        per_shard.append({"shard": s, "tiles": tiles, "pairs": pairs, "tile_kernel_ms": tile_s * 1e3,
                          "call_ms": call_s * 1e3})
        log("shard %d/%d: R %d, %d tiles, tile kernel %.3f ms, call %.3f ms" % (s, G, R, tiles, tile_s * 1e3,
                                                                             call_s * 1e3))
        if s == 0:
            avg0, R0, pairs0, tile0 = call_s, R, pairs, tile_s
    achieved = FLOP_PER_PAIR * pairs0 / tile0 / 1e12
    tile_ms = [r["tile_kernel_ms"] for r in per_shard]
    result = {
        "metric": "repulsion pair-interactions/s of one GPU's share (shard 0 of %d) at 300K nodes" % G,
        "value": pairs0 / avg0, "unit": "pair-interactions/s", "n_gpus": 1, "steps": reps,
        "warmup": max(args.warmup, 10), "ms_per_step": avg0 * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (FP64 Z and cross-tile sums)", "data": "synthetic",
        "config": {"workload": "shard_300k", "nodes": n, "shards": G, "shard": 0, "tile_rows": R0,
                   "layout": "N(0, 100 I)", "step": "tsgne_shard_repulsion (tile kernel + Z sum + row sums)"},
        "roofline": {"bound": "alu", "kernel": "k_repulse (shard 0's tiles)", "achieved": achieved,
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": measured_traffic("shard_300k", repulse_kernel_name(R0)),
                     "flop_per_launch": FLOP_PER_PAIR * pairs0,
                     "avg_launch_ms": tile0 * 1e3},
        "shards": per_shard,
        "balance_max_over_mean": max(tile_ms) / (sum(tile_ms) / len(tile_ms)),
    }
    if not args.no_cpu_baseline:
        import oracle
        T = 64 * R0
        nb = -(-n // T)
        a = np.arange(nb)
        counted = ((np.minimum(a, nb - 1 - a) % G) == 0).astype(np.uint8)
        group = (np.arange(n) // T).astype(np.int32)
        Y64 = Y.cpu().numpy().astype(np.float64)
        sizes = np.minimum(T, n - a * T)
        rng = np.random.default_rng(3)

        def counted_pairs(rows):
            k = rows // T
            per_block = np.array([(counted[np.minimum(b, a)] * sizes).sum() for b in range(nb)])
            return int((per_block[k] - counted[k]).sum())

        rows = rng.integers(0, n, 64).astype(np.int32)
        t0 = time.perf_counter()
        oracle.repulsion_terms(Y64, group=group, counted=counted, rows=rows, with_Z=False)
        dt = time.perf_counter() - t0
        m = int(min(n, max(64, 64 * args.cpu_seconds / max(dt, 1e-3))))
        rows = rng.integers(0, n, m).astype(np.int32)
        t0 = time.perf_counter()
        oracle.repulsion_terms(Y64, group=group, counted=counted, rows=rows, with_Z=False)
        dt = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": counted_pairs(rows) / dt, "unit": "pair-interactions/s",
                                  "cores": oracle.num_threads(), "kind": "oracle",
                                  "sample": "FP64 force sums of shard 0 for %d random rows (all their counted "
                                            "pairs), %.1f s" % (m, dt)}
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)
    return 0


def run_knn(args) -> int:
    """The t-SGNE neighbourhood graph G_knn,G (section 2.2, eq. (7)) of the
    300,000-node, 1,000,000-edge graph with k = 90 (three times the default
    perplexity of 30, so that calibration has more neighbours than the
    perplexity on every row that has them)."""
    import numpy as np
    import torch

    from paper_2310_11186_amd import synth, tsgne

    dev = torch.device("cuda:0")
    gi = synth.make("dcsbm300k")
    n, k = gi.n, 90
    rp, col = tsgne.tsgne_csr_from_edges(n, gi.edges)
    d_rp, d_col = torch.from_numpy(rp).to(dev), torch.from_numpy(col).to(dev)
    for _ in range(max(args.warmup, 1)):
        krp, kcol = tsgne.tsgne_knn_graph(d_rp, d_col, k)
    reps = max(args.steps, 3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        krp, kcol = tsgne.tsgne_knn_graph(d_rp, d_col, k)
    torch.cuda.synchronize()
    avg_s = (time.perf_counter() - t0) / reps
    result = {
        "metric": "G_knn,G construction, source nodes/s",
        "value": n / avg_s, "unit": "nodes/s", "n_gpus": 1, "steps": reps, "warmup": max(args.warmup, 1),
        "ms_per_step": avg_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": "knn_dcsbm300k", "nodes": n, "stored_entries": int(col.shape[0]), "k": k,
                   "knn_entries": int(kcol.shape[0]),
                   "step": "CSR check + per-source BFS to k nodes + symmetrisation (sort, unique) + CSR"},
        "roofline": None,
    }
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        oracle.knn_graph(rp, col, k)
        cpu_s = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": n / cpu_s, "unit": "nodes/s", "cores": oracle.num_threads(),
                                  "kind": "oracle", "sample": "the whole construction, %.2f s" % cpu_s}
    print(json.dumps(result), flush=True)
    return 0


def run_walks(args) -> int:
    """Random-walk P (section 2.1) of the 300,000-node, 1,000,000-edge graph:
    32 walks of 3 steps from every node."""
    import numpy as np
    import torch

    from paper_2310_11186_amd import synth, tsgne

    dev = torch.device("cuda:0")
    gi = synth.make("dcsbm300k")
    n, walks, length, seed = gi.n, 32, 3, synth.MASTER_SEED + 9
    rp, col = tsgne.tsgne_csr_from_edges(n, gi.edges)
    d_rp, d_col, d_X = (torch.from_numpy(a).to(dev) for a in (rp, col, gi.X))
    for _ in range(max(args.warmup, 1)):
        tsgne.tsgne_build_P_walks(d_rp, d_col, d_X, walks, length, seed).close()
    reps = max(args.steps, 3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g = tsgne.tsgne_build_P_walks(d_rp, d_col, d_X, walks, length, seed)
        support = g.info()[1]
        g.close()
    torch.cuda.synchronize()
    avg_s = (time.perf_counter() - t0) / reps
    steps = n * walks * length
    result = {
        "metric": "random-walk P construction, walk steps/s",
        "value": steps / avg_s, "unit": "walk-steps/s", "n_gpus": 1, "steps": reps, "warmup": max(args.warmup, 1),
        "ms_per_step": avg_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 transition sums, u64 keys", "data": "synthetic",
        "config": {"workload": "walks_dcsbm300k", "nodes": n, "stored_entries": int(col.shape[0]), "d": gi.d,
                   "walks_per_node": walks, "length": length, "support_entries": int(support),
                   "step": "CSR check + distances + transition sums + walks + sort + support CSR + graph set-up"},
        "roofline": None,
    }
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        oracle.walk_P(rp, col, gi.X, walks, length, seed)
        cpu_s = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": steps / cpu_s, "unit": "walk-steps/s", "cores": 1, "kind": "oracle",
                                  "sample": "the whole construction, %.2f s" % cpu_s}
    print(json.dumps(result), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="dcsbm300k", help="dcsbm300k, dcsbm100k, dcsbm20k, sbm2k, dcsbm1m, dcsbm3m, dcsbm_n<N> (any size), batch256, serve, sparse, "
                         "sp, walks, knn or shard")
    ap.add_argument("--requests", type=int, default=48, help="serve: number of requests in the stream")
    ap.add_argument("--qps-fractions", default="0.5,0.8,0.95", metavar="LIST",
                    help="serve: Poisson arrival rates as fractions of the saturated rate (comma list)")
    ap.add_argument("--serve-low-budget-mb", type=int, default=512, metavar="MIB",
                    help="serve: device-memory budget of the low-budget run (0 = skip it)")
    ap.add_argument("--serve-qps", type=float, default=0.0,
                    help="serve: Poisson arrival rate (req/s); skips the saturated runs")
    ap.add_argument("--serve-only", default="", choices=["", "batched", "one_at_a_time", "oldest_share"],
                    help="serve: run only this configuration at the Poisson rate")
    ap.add_argument("--serve-round-ms", type=float, default=25.0, help="serve: the server's round_ms")
    ap.add_argument("--serve-saturated-only", action="store_true", help="serve: only the saturated runs")
    ap.add_argument("--serve-requests", type=int, default=48,
                    help="default workload: requests in the serving leg (0 = skip it)")
    ap.add_argument("--shards", type=int, default=8, help="shard: GPUs the repulsion is split over")
    ap.add_argument("--sparse-nodes", type=int, default=10_000_000, help="sparse: nodes of the SBM")
    ap.add_argument("--n-iter", type=int, default=None, help="optimisation steps per layout (default: workload's)")
    ap.add_argument("--repulsion", default="auto", choices=["auto", "direct", "symmetric"])
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--precision", default="split", choices=["split", "fp32"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (scales HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only (got --gpus %d): one GPU's share of a repulsion split over N GPUs is "
              "measured by --workload shard --shards N; the cross-GPU reductions are not built" % args.gpus,
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2310_11186_amd import synth, tsgne

    if args.workload == "batch256":
        return run_batch(args)
    if args.workload == "serve":
        return run_serve(args)
    if args.workload == "sparse":
        return run_sparse(args)
    if args.workload == "sp":
        return run_sp(args)
    if args.workload == "walks":
        return run_walks(args)
    if args.workload == "knn":
        return run_knn(args)
    if args.workload == "shard":
        return run_shard(args)

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": nbytes, "launches": 5}), flush=True)
        return 0

    # serving leg of the default line: its requests are generated by worker
    # processes forked now, before this process touches the GPU
    serve_pool = request_pool(8) if (args.workload == "dcsbm300k" and args.serve_requests > 0) else None

    dev = torch.device("cuda:0")
    wl = synth.WORKLOADS.get(args.workload) or synth.Workload(
        args.workload, "DC-SBM of the given size (average degree 8, d = 32)", 1000, 250)
    n_iter = args.n_iter if args.n_iter is not None else wl.n_iter
    t_ee = min(wl.exaggeration_iters, n_iter // 4) if args.n_iter is not None else wl.exaggeration_iters
    log("generating %s" % wl.description)
    gi = synth.make(args.workload)
    rp, col = tsgne.tsgne_csr_from_edges(gi.n, gi.edges)
    d_rp = torch.from_numpy(rp).to(dev)
    d_col = torch.from_numpy(col).to(dev)
    d_X = torch.from_numpy(gi.X).to(dev)
    d_Y0 = torch.from_numpy(gi.Y0).to(dev)
    Y = torch.empty_like(d_Y0)
    rep = {"auto": tsgne.TSGNE_REPULSION_AUTO, "direct": tsgne.TSGNE_REPULSION_DIRECT,
           "symmetric": tsgne.TSGNE_REPULSION_SYMMETRIC}[args.repulsion]
    prec = tsgne.TSGNE_PREC_FP32 if args.precision == "fp32" else tsgne.TSGNE_PREC_SPLIT
    params = tsgne.tsgne_params_default(exaggeration_iters=t_ee, early_exaggeration=wl.early_exaggeration,
                                        repulsion=rep, tile_rows=args.tile_rows, precision=prec)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    def one_step(timed_graphs=None):
        g = tsgne.tsgne_build_P(d_rp, d_col, d_X, wl.perplexity, stream)
        if timed_graphs is not None:
            g.set_timing(True)
        Y.copy_(d_Y0)
        tsgne.tsgne_run(g, Y, n_iter, params, stream)
        kl = tsgne.tsgne_kl(g, Y, stream)
        if timed_graphs is not None:
            timed_graphs.append(g.timing())
        g.close()
        return kl

    for w in range(args.warmup):
        kl = one_step()
        log("warmup %d/%d done (KL %.4f)" % (w + 1, args.warmup, kl))

    timings = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kls = []
    for k in range(args.steps):
        kls.append(one_step(timings))
        log("step %d/%d done (KL %.4f, %.1f s elapsed)" % (k + 1, args.steps, kls[-1], time.perf_counter() - t0))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # The timed layouts launch each step's kernels one by one between events
    # (phase timing); a layout without timing replays captured chunks of
    # steps.  For layouts short enough that launches matter, time that too.
    replayed_ms = None
    if elapsed / args.steps < 2.0:
        reps = 5
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            one_step()
        torch.cuda.synchronize()
        replayed_ms = (time.perf_counter() - t1) / reps * 1e3
        log("layout without phase timing (captured replay): %.2f ms" % replayed_ms)

    n = gi.n
    pairs_per_iter = n * (n - 1)
    value = args.steps * n_iter * pairs_per_iter / elapsed
    quality = layout_quality(Y, gi, dev, stream)
    rep_ms = sum(t["repulsion"][0] for t in timings)
    rep_launches = sum(t["repulsion"][1] for t in timings)
    avg_rep_s = rep_ms / max(rep_launches, 1) / 1e3
    achieved_tflops = FLOP_PER_PAIR * pairs_per_iter / avg_rep_s / 1e12 if rep_launches else None
    executed_tflops = (EXECUTED_FLOP_PER_UNORDERED_PAIR * pairs_per_iter / 2 / avg_rep_s / 1e12
                       if rep_launches else None)
    phase_avg_ms = {}
    for name in tsgne.TSGNE_PHASES:
        tot = sum(t[name][0] for t in timings)
        cnt = sum(t[name][1] for t in timings)
        phase_avg_ms[name] = round(tot / cnt, 4) if cnt else None

    result = {
        "metric": ("t-SGNE pair-interactions/s at 300K nodes (% FP32 peak); served layouts/s + p99"
                   if args.workload == "dcsbm300k" else "t-SGNE pair-interactions/s (% FP32 peak)"),
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == tsgne.TSGNE_PREC_FP32 else "f32 (FP64 Z/KL/cross-tile sums)",
        "data": "synthetic",
        "config": {
            "workload": args.workload, "description": wl.description, "nodes": n,
            "edges": int(gi.edges.shape[0]), "d": gi.d, "n_iter": n_iter, "exaggeration_iters": t_ee,
            "layout_iterations": wl.n_iter,
            "perplexity": wl.perplexity, "repulsion": args.repulsion, "precision": args.precision,
            "step": "build_P + n_iter optimisation steps + KL",
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_repulse (all-pairs repulsion + Z partials)",
            "instantiation": repulse_kernel_name(tsgne.tsgne_repulsion_plan(gi.n, args.tile_rows, rep)[0],
                                                 prec == tsgne.TSGNE_PREC_SPLIT,
                                                 rep != tsgne.TSGNE_REPULSION_DIRECT),
            "achieved": achieved_tflops,
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS if achieved_tflops else None,
            "traffic": measured_traffic(args.workload, repulse_kernel_name(
                tsgne.tsgne_repulsion_plan(gi.n, args.tile_rows, rep)[0], prec == tsgne.TSGNE_PREC_SPLIT,
                rep != tsgne.TSGNE_REPULSION_DIRECT)),
            "flop_per_launch": FLOP_PER_PAIR * pairs_per_iter,
            "achieved_basis": "algorithmic: 13 flop per ordered pair over the n(n-1) ordered pairs; the symmetric "
                              "tiles evaluate each unordered pair once and credit both ordered pairs",
            "executed": {
                "tflops": executed_tflops,
                "frac_of_peak": executed_tflops / FP32_VECTOR_PEAK_TFLOPS if executed_tflops else None,
                "frac_of_nonpacked_fma_peak": (executed_tflops / FP32_NONPACKED_FMA_TFLOPS
                                               if executed_tflops else None),
                "flop_per_unordered_pair": EXECUTED_FLOP_PER_UNORDERED_PAIR,
                "source": "FP32 flop the hardware counts per unordered pair (SQ_INSTS_VALU_FLOPS_FP32 x 64 lanes, "
                          "FMA = 2; profiles/repulsion_dcsbm300k_valu.md) x n(n-1)/2 over the launch time",
            },
            "avg_launch_ms": avg_rep_s * 1e3,
            "launches": rep_launches,
        },
        "phase_avg_ms": phase_avg_ms,
        "layout_ms_replayed": replayed_ms,
        "final_kl": kls[-1] if kls else None,
        "quality": quality,
    }
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host (~%.0f s)" % args.cpu_seconds)
        result["cpu_baseline"] = cpu_baseline(gi, n_iter, t_ee, wl.perplexity, args.cpu_seconds)
    else:
        result["cpu_baseline"] = None
    if serve_pool is not None:
        log("serving leg: %d requests (generating)" % args.serve_requests)
        reqs = serve_pool.map(synth.serving_request, synth.serving_request_specs(args.serve_requests))
        serve_pool.close()
        result["serving"] = serving_leg(reqs, 500)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
