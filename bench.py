"""Benchmark: one step = the whole hot path on the R-MAT scale-24 workload.

Step (all on one HIP stream, CSR already resident in HBM):
  rebuild   validation, per-row uint64 weight prefixes, node records, and
            the 8-ary prefix trees of every row above 8 out-edges (the
            split of large nodes; it never changes results)
  pool      short walks of <= 3 steps for every node of out-degree <= 32
            (K = 64 per node)
  run       128 walks from every one of the 2^24 sources, alpha = 0.15,
            stitched at small nodes; per-source counting, digests, top-32

Prints one JSON line. `value` is walk-steps per second of the whole step
(steps = edges traversed, restarts and every step of a stitched move
included). The roofline object describes the walk kernel, timed with HIP
events the library records on the stream it launches on.
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


WALK_SOURCES = ["paper_1903_11749_amd/csrc/walk.hip", "paper_1903_11749_amd/csrc/fppr_device.hpp",
                "paper_1903_11749_amd/csrc/fppr_internal.hpp"]
PMC_SUMMARY = "profiles/k_walk_rmat24_pmc.md"


def walk_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in WALK_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counted_traffic():
    """HBM bytes per walk launch from the committed counter summary, or None
    when the walk kernel's sources changed since the counters were taken."""
    path = os.path.join(ROOT, PMC_SUMMARY)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        line = line.strip()
        if ":" in line and line.split(":", 1)[0] in ("walk_kernel_source_sha256",
                                                     "walk_traffic_bytes_per_launch"):
            k, v = line.split(":", 1)
            vals[k] = v.strip()
    if vals.get("walk_kernel_source_sha256") != walk_source_hash():
        return None
    return int(vals["walk_traffic_bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["scale24", "medium"], default="scale24")
    ap.add_argument("--cpu-sample", type=int, default=1 << 20,
                    help="sources in the oracle's timed sample (0 = skip)")
    ap.add_argument("--no-check", action="store_true", help="skip the sampled parity check")
    ap.add_argument("--hub-threshold", type=int, default=0,
                    help="rows above this many edges get a prefix tree (0 = library default)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES device-to-device 3 times (scale for byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1",
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

    if args.workload == "scale24":
        cfg = dict(synth.SCALE24)
        t0 = time.time()
        g = synth.scale24_graph()
        wname = ("rmat-scale24 (n=2^24, m=2^28, a,b,c,d=.57,.19,.19,.05, Zipf(1.2) weights "
                 "in [1,1e4]), alpha=0.15, R=128, all sources, short walks S=32 L=3 K=64, "
                 "large rows split, top-32")
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
    G = fppr.Graph(n=g.n, row_offsets=ro, col=col, w=w, hub_threshold=args.hub_threshold)
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

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    walk_ms, agg_ms, steps_total, st_last = [], [], 0, None
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record(stream)
    for i in range(args.steps):
        step()
        wm, am = prof.read()  # waits for this step's walk + aggregation events
        walk_ms.append(wm)
        agg_ms.append(am)
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

    walk_avg = float(np.mean(walk_ms))
    ab = alg_bytes(st_last)
    achieved = ab / (walk_avg / 1e3) / 1e9
    traffic = counted_traffic() if args.workload == "scale24" else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 5), "traffic": traffic,
                "kernel": "k_walk", "kernel_ms": round(walk_avg, 3),
                "alg_bytes_per_launch": ab,
                "walk_steps_per_s_kernel": round(st_last["steps"] / (walk_avg / 1e3), 1),
                "moves_per_s_kernel": round(st_last["moves"] / (walk_avg / 1e3), 1)}

    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "walk-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32/u64 integer",
        "data": "synthetic (seeded R-MAT; stands in for the paper's SNAP graphs)",
        "config": {"workload": wname, "n": g.n, "m": g.m, "R": R, "alpha": alpha, "seed": seed,
                   "topk": k, "tree_rows": info["hubs"], "small_nodes": info["small"],
                   "rows_over_4096": int((g.degrees() > 4096).sum())},
        "sources_per_s": round(sources_per_s, 1),
        "walk_stats_per_step": st_last,
        "aggregate_ms": round(float(np.mean(agg_ms)), 3),
        "wall_s": round(wall, 3),
        "roofline": roofline,
    }

    # ---- oracle: sampled parity + CPU baseline (rank 0, N = 1) ----
    if args.cpu_sample > 0:
        from oracle import oracle as O

        nthreads = max(1, min(16, os.cpu_count() or 1))
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
        result["cpu_baseline"] = {
            "value": round(cpu_steps, 1), "unit": "walk-steps/s", "cores": nthreads, "kind": "oracle",
            "sample": (f"{len(sample)} uniform random sources x {R} walks of the same workload "
                       f"(walks + counting + top-k, {t_cpu:.2f}s); short-walk pool built "
                       f"beforehand in {t_pool:.1f}s, not in the rate"),
            "sources_per_s": round(len(sample) / t_cpu, 1),
        }
        if not args.no_check:
            got_d = out.digest.cpu().numpy().view(np.uint64)[sample]
            got_k = out.topk.cpu().numpy().view(np.uint32)[sample]
            ok = bool(np.array_equal(got_d, ref.digest) and np.array_equal(got_k, ref.topk))
            result["parity_sample"] = {"sources": len(sample), "bit_exact": ok}
            if not ok:
                log("PARITY MISMATCH on the sampled sources")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
