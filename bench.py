"""Benchmark: one step = the whole hot path on the R-MAT scale-24 workload.

Step (all on one HIP stream, CSR already resident in HBM):
  rebuild   validation and the search structure of every row's weights:
            by default the guide tables (per-edge draw thresholds of the
            uint64 weight prefixes, row tables indexed by the draw's top bits
            and their child tables; one 64-byte read per weighted pick for
            almost every draw), or with --layout narrow/wide the node records
            and the prefix trees of every row above 8 out-edges (the split of
            large nodes); every layout gives the same edge for every draw
  pool      short walks of <= 3 steps for every node of out-degree <= 32
            (K = 64 per node)
  run       128 walks from every one of the 2^24 sources, alpha = 0.15,
            stitched at small nodes; per-source counting, digests, top-32

Prints one JSON line. `value` is walk-steps per second of the whole step
(steps = edges traversed, restarts and every step of a stitched move
included). The roofline object describes the walk kernel (k_walk_guide, or
k_walk for the tree layouts), timed with
HIP events the library records on the stream it launches on; in all-nodes
runs on graphs where a quarter or more of the nodes have no out-edges, the
walks from those nodes run in a coin-only kernel (k_dangling) beside it on a
second stream, reported beside the roofline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0

METRIC = "walk-steps/s + sources/s (batched vs plain, 1 GPU, bit-exact); p99 query latency"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def alg_bytes(st: dict) -> int:
    """Algorithmic bytes of the walk kernel for the counted work: per move the
    16-byte node record; per plain move ceil(log2 d) 8-byte prefix probes and
    one 4-byte column id; per stitched move one 8-byte pool entry; per walk
    one 4-byte endpoint write."""
    return (16 * st["moves"] + 8 * st["probe_log_sum"] + 4 * st["plain_moves"]
            + 8 * st["stitched_moves"] + 4 * st["walks"])


# the walk kernel of each layout: its sources and its committed counter summary
WALK_KERNELS = {
    "guide": ("k_walk_guide", ["paper_1903_11749_amd/csrc/walk_guide.hip", "paper_1903_11749_amd/csrc/guide.hpp",
                               "paper_1903_11749_amd/csrc/fppr_device.hpp",
                               "paper_1903_11749_amd/csrc/fppr_internal.hpp"],
              "profiles/k_walk_guide_rmat24_pmc.md"),
    "tree": ("k_walk", ["paper_1903_11749_amd/csrc/walk.hip", "paper_1903_11749_amd/csrc/fppr_device.hpp",
                        "paper_1903_11749_amd/csrc/fppr_internal.hpp"],
             "profiles/k_walk_rmat24_pmc.md"),
}
LAYOUT_NAMES = {"guide": 3, "narrow": 2, "wide": 1, "auto": 0}


def walk_kernel(layout: str):
    return WALK_KERNELS["guide" if layout == "guide" else "tree"]


def walk_source_hash(layout: str = "guide") -> str:
    import hashlib

    h = hashlib.sha256()
    for f in walk_kernel(layout)[1]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counted_traffic(layout: str = "guide"):
    """HBM bytes of one walk-kernel launch from the committed counter
    summary, or None when the walk kernel's sources changed since the
    counters were taken."""
    path = os.path.join(ROOT, walk_kernel(layout)[2])
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        line = line.strip()
        if ":" in line and line.split(":", 1)[0] in ("walk_kernel_source_sha256",
                                                     "walk_traffic_bytes_per_launch"):
            k, v = line.split(":", 1)
            vals[k] = v.strip()
    if vals.get("walk_kernel_source_sha256") != walk_source_hash(layout):
        return None
    return int(vals["walk_traffic_bytes_per_launch"])


BATCH_TOPK = 16
BATCH_POOLS = [dict(S=32, L=3, K=64), dict(S=16, L=2, K=32)]
BATCH_HUB_THRESHOLDS = [8, 64, 0xFFFFFFFF]
BATCH_BLOCKS_PER_CU = [0, 2]


def bench_batch(args, fppr, torch, np):
    """The 64-graph batch: autotune each graph, then time one captured replay
    of the whole batch (every graph's rebuild and pool, one walk launch, every
    graph's counting and top-k) against the same work as 64 plain per-graph
    launches in sequence; both must give bit-identical outputs. Everything,
    torch's own fills included, runs on one stream other than the null stream
    (which capture needs)."""
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        res = _bench_batch(args, fppr, torch, np, stream)
    torch.cuda.synchronize()
    return res


def _bench_batch(args, fppr, torch, np, stream):
    import collections

    import synth

    t0 = time.time()
    specs = synth.batch_specs()
    graphs = [synth.batch_graph(sp) for sp in specs]
    log(f"batch: generated {len(graphs)} graphs, {sum(g.n for g in graphs)} nodes, "
        f"{sum(g.m for g in graphs)} edges in {time.time() - t0:.1f}s")
    Gs, manifest = [], []
    t0 = time.time()
    guide = args.batch_layout == "guide"
    for sp, g in zip(specs, graphs):
        G = fppr.Graph(g, layout=LAYOUT_NAMES[args.batch_layout])
        pools = [dict(o, seed=6000 + sp["index"]) for o in BATCH_POOLS]
        r = G.autotune(sp["alpha"], sp["R"], sp["walk_seed"],
                       hub_thresholds=[0] if guide else BATCH_HUB_THRESHOLDS,
                       blocks_per_cu=BATCH_BLOCKS_PER_CU, pools=pools, stream=stream)
        Gs.append(G)
        manifest.append(dict(graph=sp["index"], n=g.n, m=g.m, alpha=sp["alpha"], R=sp["R"],
                             walk_seed=sp["walk_seed"], hub_threshold=r["hub_threshold"],
                             blocks_per_cu=r["blocks_per_cu"], pool=r["pool_opts"],
                             est_ms=round(r["est_ms"], 4), plain_est_ms=round(r["plain_est_ms"], 4)))
    tune_s = time.time() - t0
    log(f"batch: tuned {len(Gs)} graphs in {tune_s:.1f}s")
    width = collections.Counter(m["blocks_per_cu"] for m in manifest).most_common(1)[0][0]
    items = [dict(graph=G, alpha=sp["alpha"], R=sp["R"], seed=sp["walk_seed"], topk=BATCH_TOPK,
                  stitch=m["pool"] is not None, sources=None)
             for G, sp, m in zip(Gs, specs, manifest)]
    B = fppr.Batch(items, counts=False, digests=True, stats=True, rebuild=True, blocks_per_cu=width)
    B.capture(stream)

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(max(1, args.warmup)):
        B.launch(stream)
    B.check(stream)
    steps, ms = 0, []
    for i in range(args.steps):
        B.stats.zero_()
        e0.record(stream)
        B.launch(stream)
        e1.record(stream)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
        steps = B.stats_dict()["steps"]
    B.check(stream)
    walks = B.stats_dict()["walks"]
    batch_ms = float(np.median(ms))
    log(f"batch: captured replay {batch_ms:.1f} ms (median of {len(ms)})")

    # the same work as plain launches, one graph after the other
    plain = []
    for G, it in zip(Gs, items):
        p = fppr.make_params(it["alpha"], it["R"], it["seed"], BATCH_TOPK, it["stitch"], counts=False,
                             digests=True, stats=False,
                             blocks_per_cu=manifest[len(plain)]["blocks_per_cu"])
        ws = torch.empty((fppr.fppr_plan(G, p, G.n) + 7) // 8, dtype=torch.int64, device="cuda")
        out = fppr.alloc_outputs(G.n, it["R"], BATCH_TOPK, counts=False, digests=True, stats=False)
        plain.append((G, p, ws, out))

    def plain_step():
        for G, p, ws, out in plain:
            G.rebuild(stream)
            fppr.fppr_run(G, p, None, G.n, ws, out, stream)

    for _ in range(max(1, args.warmup)):
        plain_step()
    torch.cuda.synchronize()
    pms = []
    for i in range(args.steps):
        e0.record(stream)
        plain_step()
        e1.record(stream)
        e1.synchronize()
        pms.append(e0.elapsed_time(e1))
    plain_ms = float(np.median(pms))
    log(f"batch: 64 plain launches {plain_ms:.1f} ms (median of {len(pms)})")
    for G, p, ws, out in plain:
        fppr.fppr_run_check(ws, stream)
        G.check(stream)
    same = all(torch.equal(a.digest, b[3].digest) and torch.equal(a.topk, b[3].topk)
               for a, b in zip(B.outputs, plain))

    # oracle on the smallest graphs
    from oracle import oracle as O

    small = sorted(range(len(specs)), key=lambda i: specs[i]["n"])[:4]
    oracle_ok = True
    for i in small:
        og = O.Graph.from_csr(graphs[i])
        pool = None
        if manifest[i]["pool"] is not None:
            po = manifest[i]["pool"]
            pool = O.Pool(og, S=po["S"], L=po["L"], K=po["K"], alpha=specs[i]["alpha"], seed=po["seed"])
        ref = O.run(og, specs[i]["alpha"], specs[i]["R"], specs[i]["walk_seed"], topk=BATCH_TOPK,
                    pool=pool, want_counts=False)
        got = B.outputs[i]
        oracle_ok &= bool(np.array_equal(got.digest.cpu().numpy().view(np.uint64), ref.digest)
                          and np.array_equal(got.topk.cpu().numpy().view(np.uint32), ref.topk))
    # and a stratified sample of the rest: every 7th graph by size (large,
    # autotuned, stitched ones included), 1,024 random sources each
    rest = sorted(range(len(specs)), key=lambda i: specs[i]["n"])[4::7]
    sampled_ok, sampled_graphs, sampled_stitched = True, 0, 0
    rs = np.random.default_rng(4242)
    for i in rest:
        og = O.Graph.from_csr(graphs[i])
        pool = None
        if manifest[i]["pool"] is not None:
            po = manifest[i]["pool"]
            pool = O.Pool(og, S=po["S"], L=po["L"], K=po["K"], alpha=specs[i]["alpha"], seed=po["seed"])
            sampled_stitched += 1
        src = np.sort(rs.choice(graphs[i].n, min(1024, graphs[i].n), replace=False)).astype(np.uint32)
        ref = O.run(og, specs[i]["alpha"], specs[i]["R"], specs[i]["walk_seed"], sources=src, topk=BATCH_TOPK,
                    pool=pool, want_counts=False)
        got = B.outputs[i]
        sampled_ok &= bool(np.array_equal(got.digest.cpu().numpy().view(np.uint64)[src], ref.digest)
                           and np.array_equal(got.topk.cpu().numpy().view(np.uint32)[src], ref.topk))
        sampled_graphs += 1
    log(f"batch: oracle on the 4 smallest graphs {oracle_ok}, on 1024 sources of {sampled_graphs} more "
        f"({sampled_stitched} stitched) {sampled_ok}")
    n_src = sum(g.n for g in graphs)
    lib_manifest = B.manifest()
    if args.manifest:
        with open(args.manifest, "w") as fh:
            json.dump(dict(tuner=manifest, batch=lib_manifest), fh, indent=1)
    res = {
        "workload": ("64 directed Chung-Lu graphs, n log-uniform in [1e3, 1e6], mean degree U[8,24], "
                     "exponent U[2.1,2.5], weights U{1..255}, alpha in {.1,.15,.2}, R in {64,256}, "
                     f"all sources, top-{BATCH_TOPK}"),
        "graphs": len(graphs), "sources": n_src, "walks": walks, "walk_steps": steps,
        "batched_ms": round(batch_ms, 3), "plain_ms": round(plain_ms, 3),
        "batched_walk_steps_per_s": round(steps / (batch_ms / 1e3), 1),
        "plain_walk_steps_per_s": round(steps / (plain_ms / 1e3), 1),
        "batched_sources_per_s": round(n_src / (batch_ms / 1e3), 1),
        "plain_sources_per_s": round(n_src / (plain_ms / 1e3), 1),
        "speedup": round(plain_ms / batch_ms, 3),
        "bit_exact_vs_plain": bool(same), "oracle_bit_exact_smallest4": bool(oracle_ok),
        "oracle_bit_exact_sampled": {"graphs": sampled_graphs, "stitched_graphs": sampled_stitched,
                                     "sources_each": 1024, "bit_exact": bool(sampled_ok)},
        "tuning_s": round(tune_s, 2),
        "tuned": {"stitched_graphs": sum(m["pool"] is not None for m in manifest),
                  "hub_thresholds": dict(collections.Counter(str(m["hub_threshold"]) for m in manifest)),
                  "launch_blocks_per_cu": width},
    }
    B.close()
    for G in Gs:
        G.close()
    return res


SERVE_TOPK = 64
SERVE_ALPHA = 0.15


def _serve_run(fppr, G, queries, mode, times=None, stitch=True, first_counted=0, **kw):
    """Submits `queries` (at their arrival offsets in `times`, seconds, or all
    at once) and collects every result. Returns (results by query, the
    library's latency statistics over queries first_counted.., makespan s,
    server stats)."""
    import collections

    import numpy as np

    S = fppr.Server(G, mode=mode, **kw)
    t0 = time.perf_counter()
    ids = []
    outstanding = collections.deque()
    results = {}

    def drain(block=False):
        while outstanding:
            qi, qid = outstanding[0]
            r = S.wait(qid) if block else S.poll(qid)
            if r is None:
                return
            results[qi] = r
            outstanding.popleft()

    for qi, q in enumerate(queries):
        if times is not None:
            due = t0 + times[qi]
            while True:
                now = time.perf_counter()
                if now >= due:
                    break
                drain()
                if due - now > 0.0005:
                    time.sleep(min(0.0005, due - now - 0.0003))
        qid = S.submit(q["sources"], q["R"], SERVE_ALPHA, q["seed"], SERVE_TOPK, stitch)
        ids.append(qid)
        outstanding.append((qi, qid))
        drain()
    drain(block=True)
    st = S.stats()
    lat = S.latency(first_id=ids[first_counted])  # ids grow in submission order
    S.close()
    sub = np.array([results[i][2]["submit_ns"] for i in range(len(queries))], dtype=np.float64)
    done = np.array([results[i][2]["done_ns"] for i in range(len(queries))], dtype=np.float64)
    makespan = (done.max() - sub.min()) / 1e9
    return results, lat, makespan, st


def bench_serve(args, fppr, torch, G, n_nodes, oracle_pool=None, oracle_graph=None):
    """Continuous-batching server vs FIFO plain launches on the resident
    scale-24 graph and pool, at the same Poisson arrival rate."""
    import numpy as np

    import synth

    torch.cuda.synchronize()
    nq, warm = args.serve_queries, args.serve_warmup
    base = synth.poisson_queries(n_nodes, nq + warm, qps=1.0, seed=5000)
    queries = [dict(sources=q["sources"], R=q["R"], seed=q["seed"]) for q in base]
    unit_times = np.array([q["arrival"] for q in base])  # arrivals at 1 query/s
    kw = dict(max_requests=64, memory_bytes=24 << 30, host_bytes=2 << 30, slice_walks=args.slice_walks)
    # saturation: everything submitted at once (closed burst)
    burst = queries[:args.serve_burst]
    _, _, fifo_span, _ = _serve_run(fppr, G, burst, "fifo", **kw)
    _, _, cont_span, _ = _serve_run(fppr, G, burst, "continuous", **kw)
    fifo_sat, cont_sat = len(burst) / fifo_span, len(burst) / cont_span
    qps = 0.9 * fifo_sat
    log(f"serve: saturation fifo {fifo_sat:.1f} q/s, continuous {cont_sat:.1f} q/s; open loop at {qps:.1f} q/s")
    times = unit_times / qps
    out = {}
    res_by_mode = {}
    for mode in ("fifo", "continuous"):
        res, lat, span, st = _serve_run(fppr, G, queries, mode, times=times, first_counted=warm, **kw)
        out[mode] = {"p50_ms": round(lat["p50_ms"], 3), "p99_ms": round(lat["p99_ms"], 3),
                     "mean_ms": round(lat["mean_ms"], 3), "max_ms": round(lat["max_ms"], 3),
                     "latency_from": "fppr_server_latency over the queries after the warm-up",
                     "counted_queries": int(lat["count"]), "counted_qps": round(lat["qps"], 2),
                     "queries_per_s": round(len(queries) / span, 2),
                     "sources_per_s": round(sum(q["sources"].size for q in queries) / span, 1),
                     "walk_steps_per_s": round(st["walk_stats"]["steps"] / span, 1),
                     "walks": int(st["walk_stats"]["walks"]), "slices": int(st["slices"]),
                     "peak_in_flight": int(st["peak_in_flight"])}
        res_by_mode[mode] = res
        log(f"serve {mode}: p50 {out[mode]['p50_ms']} ms, p99 {out[mode]['p99_ms']} ms, "
            f"{out[mode]['queries_per_s']} q/s")
    same = all(np.array_equal(res_by_mode["fifo"][i][0], res_by_mode["continuous"][i][0]) and
               np.array_equal(res_by_mode["fifo"][i][1], res_by_mode["continuous"][i][1])
               for i in range(len(queries)))
    # 200 queries stratified by walk budget (every budget decile, small and
    # large R, few and many sources): each rerun alone with fppr_run, and in
    # the oracle on two of its sources (sources are independent, so a
    # source's row is exact on its own) plus every source of the 3 smallest
    order = sorted(range(len(queries)), key=lambda i: queries[i]["sources"].size * queries[i]["R"])
    pick = [order[int(j)] for j in np.linspace(0, len(order) - 1, min(200, len(order)))]
    alone_ok = True
    for i in pick:
        q = queries[i]
        o = fppr.run(G, SERVE_ALPHA, q["R"], q["seed"], sources=q["sources"], topk=SERVE_TOPK, stitch=True,
                     counts=False, stats=False)
        torch.cuda.synchronize()
        alone_ok &= bool(np.array_equal(o.topk.cpu().numpy().view(np.uint32), res_by_mode["continuous"][i][0])
                         and np.array_equal(o.digest.cpu().numpy().view(np.uint64),
                                            res_by_mode["continuous"][i][1]))
    oracle_ok, oracle_walks = None, 0
    if oracle_pool is not None:
        from oracle import oracle as O

        rng = np.random.default_rng(17)
        oracle_ok = True
        for i in list(pick) + order[:3]:
            q = queries[i]
            rows = (np.arange(q["sources"].size) if i in order[:3]
                    else np.unique(rng.choice(q["sources"].size, min(2, q["sources"].size), replace=False)))
            ref = O.run(oracle_graph, SERVE_ALPHA, q["R"], q["seed"], sources=q["sources"][rows], topk=SERVE_TOPK,
                        pool=oracle_pool, want_counts=False)
            oracle_walks += rows.size * q["R"]
            oracle_ok &= bool(np.array_equal(res_by_mode["continuous"][i][0][rows], ref.topk)
                              and np.array_equal(res_by_mode["continuous"][i][1][rows], ref.digest))
        log(f"serve: {len(pick)} queries alone {alone_ok}, oracle {oracle_ok} ({oracle_walks} walks)")
    return {
        "workload": (f"resident rmat-scale24 graph + short-walk pool; {nq} Poisson queries after {warm} "
                     "warm-up, 1..1024 uniform sources each, R log-uniform in [1e3, 1e5], alpha 0.15, "
                     "top-64, seed = query id"),
        "qps": round(qps, 2), "fifo_saturation_qps": round(fifo_sat, 2),
        "continuous_saturation_qps": round(cont_sat, 2),
        "fifo": out["fifo"], "continuous": out["continuous"],
        "p99_speedup": round(out["fifo"]["p99_ms"] / out["continuous"]["p99_ms"], 3),
        "bit_exact_fifo_vs_continuous": bool(same),
        "replay": {"queries": len(pick), "stratified_by": "walk budget n_sources x R",
                   "bit_exact_alone": bool(alone_ok),
                   "oracle": ("two random sources of each of the 200 queries and every source of the 3 "
                              "smallest, full R"),
                   "oracle_walks": int(oracle_walks), "oracle_bit_exact": oracle_ok},
    }


PAPER_REFERENCE = {
    "absolute_numbers": None,
    "note": ("the paper prints no absolute running times or rates for this path (its result "
             "plots are not in the text), so vs_baseline is null; its relative figures, "
             "with the hardware they were measured on:"),
    "hardware": ("51 machines (1 master + 50 workers), each a 12-core Intel Xeon E5-2670 with "
                 "16 GB RAM, Spark 2.0 / Scala; 13 SNAP graphs of 5K-68M nodes and 29K-2.6B edges; "
                 "eps = delta = alpha = 0.5, p_f = 1/n; mean of 3 runs, 24 h cutoff"),
    "relative": {
        "vs Doubling and GraphX-PPR": "up to two orders of magnitude faster (Sec. 5)",
        "big moves": "about 1.5x (Fig. 5(b))",
        "alias tree": "about 1.0x, but needed for Twitter (d_max about 3.0M)",
        "all three optimisations": "up to 2x",
        "accuracy vs Doubling": "NDCG up to +21 %, MAP up to +19 % at top-1000 (Sec. 5.2)",
    },
}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def ablation(args, fppr, torch, np, g, ro, col, w, cfg, st_cfg, stream, value, ms_per_step):
    """The paper's optimisation ablation (Fig. 5(b)) on this path: the same
    step without the short-walk pool (plain walks), and with the tree layout
    in place of the guide tables, with and without prefix trees (rows then
    binary-searched over their leaf blocks), each as a graph of its own on
    the same borrowed CSR, timed like the main step."""
    alpha, R, seed, k = cfg["alpha"], cfg["R"], cfg["seed"], cfg["topk"]
    head = f"stitched_{args.layout}"
    variants = {head: {"ms_per_step": round(ms_per_step, 3), "walk_steps_per_s": round(value, 1)}}
    runs = [(f"plain_{args.layout}", False, args.layout, 0)] if args.layout == "guide" else []
    runs += [("stitched_trees", True, "narrow", 0), ("plain_trees", False, "narrow", 0),
             ("stitched_no_trees", True, "narrow", 0xFFFFFFFF), ("plain_no_trees", False, "narrow", 0xFFFFFFFF)]
    runs = [r for r in runs if r[0] not in variants]
    for name, stitch, layout, H in runs:
        G = fppr.Graph(n=g.n, row_offsets=ro, col=col, w=w, hub_threshold=H, layout=LAYOUT_NAMES[layout])
        if stitch:
            G.build_pool(S=st_cfg["S"], L=st_cfg["L"], K=st_cfg["K"], alpha=alpha, seed=st_cfg["seed"])
        p = fppr.make_params(alpha, R, seed, k, stitch=stitch, counts=False, digests=True, stats=True)
        ws = torch.empty((fppr.fppr_plan(G, p, g.n) + 7) // 8, dtype=torch.int64, device="cuda")
        o = fppr.alloc_outputs(g.n, R, k, counts=False, digests=True, stats=True)

        def one():
            o.stats.zero_()
            G.rebuild(stream)
            fppr.fppr_run(G, p, None, g.n, ws, o, stream)

        for _ in range(2):
            one()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(3):
            one()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        st = o.stats_dict()
        variants[name] = {"ms_per_step": round(ms, 3), "walk_steps_per_s": round(st["steps"] / (ms / 1e3), 1),
                          "moves": st["moves"], "steps": st["steps"]}
        log(f"ablation {name}: {ms:.1f} ms per step")
        del ws, o
        G.close()
        torch.cuda.synchronize()
    base = variants[head]["ms_per_step"]
    for v in variants.values():
        v["slowdown_vs_full"] = round(v["ms_per_step"] / base, 3)
    return {"what": ("the scale-24 step without the short-walk pool (plain walks: results differ, "
                     "same law), with prefix trees in place of guide tables and without either "
                     "(identical results), like Fig. 5(b)"),
            "variants": variants}


def full_parity(args, g, G, out, cfg, st_cfg):
    """Every source of the workload against the oracle (digest and top-k of
    each), in blocks of sources logged as they finish."""
    import numpy as np

    from oracle import oracle as O

    alpha, R, seed, k = cfg["alpha"], cfg["R"], cfg["seed"], cfg["topk"]
    nthreads = max(1, min(16, os.cpu_count() or 1))
    og = O.Graph.from_csr(g)
    pool = None
    t0 = time.perf_counter()
    if st_cfg:
        pool = O.Pool(og, S=st_cfg["S"], L=st_cfg["L"], K=st_cfg["K"], alpha=alpha, seed=st_cfg["seed"],
                      nthreads=nthreads)
        log(f"full parity: oracle pool {time.perf_counter() - t0:.1f}s")
        ok_pool = bool(np.array_equal(G.export_pool(), pool.entries()))
        log(f"full parity: pool equal entry for entry: {ok_pool}")
    else:
        ok_pool = None
    dig = out.digest.cpu().numpy().view(np.uint64)
    top = out.topk.cpu().numpy().view(np.uint32)
    block = 1 << 20
    bad, steps, moves = 0, 0, 0
    t0 = time.perf_counter()
    for b0 in range(0, g.n, block):
        src = np.arange(b0, min(g.n, b0 + block), dtype=np.uint32)
        ref = O.run(og, alpha, R, seed, sources=src, topk=k, pool=pool, nthreads=nthreads, want_counts=False)
        bad += int(np.count_nonzero((ref.digest != dig[src]) | np.any(ref.topk != top[src], axis=(1, 2))))
        steps += ref.stats["steps"]
        moves += ref.stats["moves"]
        log(f"full parity: sources {b0}..{src[-1]} done, {bad} differing so far, "
            f"{time.perf_counter() - t0:.0f}s")
    gpu = out.stats_dict()
    res = {"full_parity": {"workload": "rmat-scale24 all sources" if st_cfg else "all sources",
                           "sources": int(g.n), "walks": int(g.n) * R, "differing_sources": bad,
                           "pool_equal": ok_pool, "oracle_steps": int(steps), "gpu_steps": gpu["steps"],
                           "oracle_moves": int(moves), "gpu_moves": gpu["moves"],
                           "oracle_seconds": round(time.perf_counter() - t0, 1), "oracle_threads": nthreads}}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["scale24", "medium", "batch", "serve"], default="scale24")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-graph batched-vs-plain comparison of the default run")
    ap.add_argument("--manifest", default="", help="write the batch autotuner's choices here (JSON)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving comparison of the default run")
    ap.add_argument("--serve-queries", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-burst", type=int, default=300, help="queries of the saturation bursts")
    ap.add_argument("--slice-walks", type=int, default=1 << 26, help="walks per continuous-batching slice")
    ap.add_argument("--cpu-sample", type=int, default=1 << 20,
                    help="sources in the oracle's timed sample (0 = skip)")
    ap.add_argument("--no-check", action="store_true", help="skip the sampled parity check")
    ap.add_argument("--hub-threshold", type=int, default=0,
                    help="rows above this many edges get a prefix tree (0 = library default)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES device-to-device 3 times (scale for byte counters)")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the runs without stitching and without prefix trees")
    ap.add_argument("--cpu-sample-1t", type=int, default=1 << 14,
                    help="sources of the oracle's one-thread timing (0 = skip)")
    ap.add_argument("--layout", choices=sorted(LAYOUT_NAMES), default="guide",
                    help="search structure of the weighted pick (every layout gives identical results)")
    ap.add_argument("--batch-layout", choices=sorted(LAYOUT_NAMES), default="guide")
    ap.add_argument("--full-parity", action="store_true",
                    help="one step, then every source checked against the oracle (scale 24: minutes)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1903_11749_amd import fppr

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    fppr.lib()

    if args.calibrate_copy:
        nb = args.calibrate_copy // 4 * 4
        src = torch.ones(nb // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nb, "copies": 3}), flush=True)
        return

    if args.workload == "batch":
        res = bench_batch(args, fppr, torch, np)
        print(json.dumps({
            "metric": METRIC, "value": res["batched_walk_steps_per_s"], "unit": "walk-steps/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["batched_ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "u32/u64 integer", "data": "synthetic (seeded Chung-Lu graphs)",
            "config": {"workload": res["workload"]}, "batched": res}), flush=True)
        return

    if args.workload in ("scale24", "serve"):
        cfg = dict(synth.SCALE24)
        t0 = time.time()
        g = synth.scale24_graph()
        picks = ("weighted picks through guide tables (row tables indexed by the draw, child "
                 "tables where edges crowd; the workload's 4096-edge hub split is subsumed: every "
                 "row costs about one 64-byte read per pick, results identical)"
                 if args.layout == "guide" else
                 "large rows split (prefix trees above 8 edges: the workload's 4096-edge hub "
                 "threshold gives identical results, 8 measured faster)")
        wname = ("rmat-scale24 (n=2^24, m=2^28, a,b,c,d=.57,.19,.19,.05, Zipf(1.2) weights "
                 "in [1,1e4]), alpha=0.15, R=128, all sources, short walks S=32 L=3 K=64, "
                 f"{picks}, top-32")
    else:
        cfg = dict(synth.MEDIUM)
        cfg["hub_threshold"] = 4096
        t0 = time.time()
        g = synth.medium_graph()
        wname = ("rmat-scale20 (n=2^20, m=2^24, Zipf(1.5) weights in [1,1000]), alpha=0.15, "
                 "R=200, all sources, plain walks, top-32")
    log(f"generated {g.n} nodes {g.m} edges in {time.time() - t0:.1f}s")
    alpha, R, seed, k = cfg["alpha"], cfg["R"], cfg["seed"], cfg["topk"]
    st_cfg = cfg.get("stitch")

    stream = torch.cuda.current_stream()
    ro = torch.from_numpy(g.row_offsets.view(np.int64)).cuda()
    col = torch.from_numpy(g.col.view(np.int32)).cuda()
    w = torch.from_numpy(g.w.view(np.int32)).cuda()
    torch.cuda.synchronize()
    G = fppr.Graph(n=g.n, row_offsets=ro, col=col, w=w, hub_threshold=args.hub_threshold,
                   layout=LAYOUT_NAMES[args.layout])
    if st_cfg:
        G.build_pool(S=st_cfg["S"], L=st_cfg["L"], K=st_cfg["K"], alpha=alpha, seed=st_cfg["seed"])
    info = G.info()
    log(f"graph on device: {info}")

    params = fppr.make_params(alpha, R, seed, k, stitch=bool(st_cfg), counts=False, digests=True,
                              stats=True)
    n_src = g.n
    ws_bytes = fppr.fppr_plan(G, params, n_src)
    ws = torch.empty((ws_bytes + 7) // 8, dtype=torch.int64, device="cuda")
    out = fppr.alloc_outputs(n_src, R, k, counts=False, digests=True, stats=True)
    prof = fppr.Profile()
    out.profile = prof

    def step():
        out.stats.zero_()
        G.rebuild(stream)  # prefixes, records, hubs (+ pool when built)
        fppr.fppr_run(G, params, None, n_src, ws, out, stream)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    G.check(stream)
    if args.full_parity:
        full_parity(args, g, G, out, cfg, st_cfg)
        return

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    walk_ms, agg_ms, kern_ms, coin_ms, steps_total, st_last = [], [], [], [], 0, None
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record(stream)
    for i in range(args.steps):
        step()
        wm, am = prof.read()  # waits for this step's walk + aggregation events
        km, cm = prof.read_walk()
        walk_ms.append(wm)
        agg_ms.append(am)
        kern_ms.append(km)
        coin_ms.append(cm)
        st_last = out.stats_dict()
        steps_total += st_last["steps"]
        log(f"step {i + 1}/{args.steps}: walk {wm:.1f} ms, aggregate {am:.1f} ms")
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms_total = e0.elapsed_time(e1)
    ms_per_step = ms_total / args.steps
    value = steps_total / (ms_total / 1e3)
    sources_per_s = n_src * args.steps / (ms_total / 1e3)

    # Work of the coin-only kernel, counted apart from the walk kernel's: the
    # same walks (keys depend on source, walk and move only) from an untimed
    # run over the nodes without out-edges as an explicit source list.
    kern_avg, coin_avg = float(np.mean(kern_ms)), float(np.mean(coin_ms))
    st_coin = {"walks": 0, "moves": 0}
    dang = np.flatnonzero(g.degrees() == 0).astype(np.uint32)
    split = dang.size > 0 and dang.size * 4 >= g.n  # the library's rule for the coin-only kernel
    if split:
        o = fppr.run(G, alpha, R, seed, sources=dang, topk=0, stitch=bool(st_cfg), counts=False,
                     digests=False, stats=True, stream=stream)
        st_coin = o.stats_dict()
        del o
        assert st_coin["plain_moves"] == 0 and st_coin["stitched_moves"] == 0
    st_walk = dict(st_last)
    for key in ("walks", "moves", "steps", "dangling_moves"):
        st_walk[key] -= st_coin.get(key, 0)
    ab = alg_bytes(st_walk)
    achieved = ab / (kern_avg / 1e3) / 1e9
    traffic = counted_traffic(args.layout) if args.workload in ("scale24", "serve") else None
    kname = walk_kernel(args.layout)[0]
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 5), "traffic": traffic,
                "kernel": kname, "kernel_ms": round(kern_avg, 3), "alg_bytes_per_launch": ab,
                "traffic_GBps": round(traffic / (kern_avg / 1e3) / 1e9, 1) if traffic else None,
                "walk_steps_per_s_kernel": round(st_walk["steps"] / (kern_avg / 1e3), 1),
                "moves_per_s_kernel": round(st_walk["moves"] / (kern_avg / 1e3), 1)}
    coin_only = None
    if split:
        coin_only = {"kernel": "k_dangling", "stream": f"the graph's side stream, beside {kname}",
                     "ms_after_walk_kernel": round(coin_avg, 3), "walks": st_coin["walks"],
                     "moves": st_coin["moves"], "bound": "alu (one Philox4x32-10 block per move)"}

    graph_steps = steps_total / args.steps - st_coin.get("steps", 0)
    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "walk-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32/u64 integer",
        "data": "synthetic (seeded R-MAT; stands in for the paper's SNAP graphs)",
        "config": {"workload": wname, "n": g.n, "m": g.m, "R": R, "alpha": alpha, "seed": seed,
                   "topk": k, "layout": args.layout, "tree_rows": info["hubs"], "small_nodes": info["small"],
                   "rows_over_4096": int((g.degrees() > 4096).sum())},
        "sources_per_s": round(sources_per_s, 1),
        "graph_steps_per_s": round(graph_steps / (ms_per_step / 1e3), 1),
        "graph_steps_note": ("steps that read the graph (those of the walk kernel; the coin-only "
                             "restart steps of the walks from nodes without out-edges excluded), "
                             "over the whole step time"),
        "walk_stats_per_step": st_last,
        "aggregate_ms": round(float(np.mean(agg_ms)), 3),
        "walk_phase_ms": round(float(np.mean(walk_ms)), 3),
        "rebuild_and_pool_ms": round(ms_per_step - float(np.mean(walk_ms)) - float(np.mean(agg_ms)), 3),
        "wall_s": round(wall, 3),
        "roofline": roofline,
        "coin_only": coin_only,
        "paper_reference": PAPER_REFERENCE,
    }
    if args.workload == "scale24" and not args.no_ablation:
        result["ablation"] = ablation(args, fppr, torch, np, g, ro, col, w, cfg, st_cfg, stream, value,
                                      ms_per_step)

    # ---- oracle: sampled parity + CPU baseline (rank 0, N = 1) ----
    og = pool = None
    if args.cpu_sample > 0:
        from oracle import oracle as O

        ncpu = os.cpu_count() or 1
        nthreads = max(1, min(16, ncpu))
        og = O.Graph.from_csr(g)
        pool = None
        t_pool = 0.0
        if st_cfg:
            tp = time.perf_counter()
            pool = O.Pool(og, S=st_cfg["S"], L=st_cfg["L"], K=st_cfg["K"], alpha=alpha,
                          seed=st_cfg["seed"], nthreads=nthreads)
            t_pool = time.perf_counter() - tp
            log(f"oracle pool {t_pool:.1f}s")
        rng = np.random.Generator(np.random.Philox(777))
        sample = np.sort(rng.choice(g.n, min(args.cpu_sample, g.n), replace=False)).astype(np.uint32)
        tc = time.perf_counter()
        ref = O.run(og, alpha, R, seed, sources=sample, topk=k, pool=pool, nthreads=nthreads,
                    want_counts=False)
        t_cpu = time.perf_counter() - tc
        cpu_steps = ref.stats["steps"] / t_cpu
        log(f"oracle sample {t_cpu:.1f}s ({cpu_steps:.3g} steps/s)")
        one = None
        if args.cpu_sample_1t > 0:
            s1 = sample[:: max(1, len(sample) // args.cpu_sample_1t)][: args.cpu_sample_1t]
            t1 = time.perf_counter()
            r1 = O.run(og, alpha, R, seed, sources=s1, topk=k, pool=pool, nthreads=1, want_counts=False)
            t1 = time.perf_counter() - t1
            one = {"walk_steps_per_s": round(r1.stats["steps"] / t1, 1), "sources": int(len(s1)),
                   "seconds": round(t1, 3)}
            log(f"oracle one thread {t1:.1f}s ({r1.stats['steps'] / t1:.3g} steps/s)")
        # the whole workload on the host at this rate, with the pool build
        # (both are in the GPU's step)
        whole_s = t_pool + t_cpu * g.n / len(sample)
        result["cpu_baseline"] = {
            "value": round(cpu_steps, 1), "unit": "walk-steps/s", "cores": nthreads, "kind": "oracle",
            "sample": (f"{len(sample)} uniform random sources x {R} walks of the same workload "
                       f"(walks + counting + top-k, {t_cpu:.2f}s); short-walk pool built "
                       f"beforehand in {t_pool:.1f}s, not in the rate"),
            "sources_per_s": round(len(sample) / t_cpu, 1),
            "host": {"nproc": ncpu, "cpu_model": cpu_model(), "threads_used": nthreads},
            "one_thread": one,
            "pool_build_s": round(t_pool, 2),
            "whole_step_estimate": {
                "seconds": round(whole_s, 1),
                "walk_steps_per_s": round(steps_total / args.steps / whole_s, 1),
                "how": ("pool build + the sample's time scaled to all sources, i.e. the same work as "
                        "one GPU step (rebuild aside)"),
                "gpu_step_ms": round(ms_per_step, 3),
            },
        }
        if not args.no_check:
            got_d = out.digest.cpu().numpy().view(np.uint64)[sample]
            got_k = out.topk.cpu().numpy().view(np.uint32)[sample]
            ok = bool(np.array_equal(got_d, ref.digest) and np.array_equal(got_k, ref.topk))
            result["parity_sample"] = {"sources": len(sample), "bit_exact": ok}
            if not ok:
                log("PARITY MISMATCH on the sampled sources")
    if args.workload in ("scale24", "serve") and not args.no_serve:
        result["serving"] = bench_serve(args, fppr, torch, G, g.n, oracle_pool=pool, oracle_graph=og)
    if args.workload == "scale24" and not args.no_batch:
        result["batched"] = bench_batch(args, fppr, torch, np)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
