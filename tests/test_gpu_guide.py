"""The guide-table layout (FPPR_LAYOUT_GUIDE): the same edge for every draw as
the flat search of Sec. 2.1, so every run is bit-identical to the oracle and
to the tree layouts: plain and stitched walks, pools, statistics (including
the sum of ceil(log2 deg) over picks), rows of every weight shape (child
tables several levels deep), row totals above 2^32, rebuilds of a borrowed
CSR, source lists, the per-lane-key form (many descriptors on one graph)
and the scale-24 workload in the benchmark's launch configuration."""
import sys

import numpy as np
import pytest

import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fp():
    import torch

    from paper_1903_11749_amd import fppr

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    fppr.lib()
    return fppr


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def u64(t):
    return t.cpu().numpy().view(np.uint64)


def compare(out, ref, k, counts=True, sample=None):
    import torch

    torch.cuda.synchronize()
    rows = slice(None) if sample is None else np.asarray(sample)
    if counts and ref.counts is not None:
        assert np.array_equal(u32(out.n_distinct)[rows], ref.n_distinct)
        assert np.array_equal(u32(out.counts)[rows], ref.counts)
    if k:
        assert np.array_equal(u32(out.topk)[rows], ref.topk)
    assert np.array_equal(u64(out.digest)[rows], ref.digest)


def stats_equal(out, ref_stats):
    st = out.stats_dict()
    for key in ("walks", "moves", "steps", "capped", "dangling_moves", "plain_moves",
                "stitched_moves", "probe_log_sum"):
        assert st[key] == ref_stats[key], (key, st[key], ref_stats[key])


def check_all(fp, g, alpha, R, seed, k, pool_opts=None, narrow_too=True):
    """Every source, plain and (with pool_opts) stitched: guide = oracle
    (counts, top-k, digests, statistics, pool) = narrow layout."""
    G = fp.Graph(g, layout=fp.FPPR_LAYOUT_GUIDE)
    assert G.layout() == fp.FPPR_LAYOUT_GUIDE
    og = O.Graph.from_csr(g)
    Gn = fp.Graph(g) if narrow_too else None
    for stitch in ((False, True) if pool_opts else (False,)):
        pool = None
        if stitch:
            G.build_pool(alpha=alpha, **pool_opts)
            pool = O.Pool(og, alpha=alpha, **pool_opts)
            assert np.array_equal(G.export_pool(), pool.entries())
            if Gn is not None:
                Gn.build_pool(alpha=alpha, **pool_opts)
        out = fp.run(G, alpha, R, seed, topk=k, stitch=stitch, counts=True, stats=True)
        ref = O.run(og, alpha, R, seed, topk=k, pool=pool)
        compare(out, ref, k)
        stats_equal(out, ref.stats)
        if Gn is not None:
            outn = fp.run(Gn, alpha, R, seed, topk=k, stitch=stitch, counts=True, stats=True)
            compare(outn, ref, k)
    G.close()
    if Gn is not None:
        Gn.close()


def test_small_all_sources(fp):
    say("case: guide layout, small graph, plain and stitched")
    check_all(fp, synth.small_graph(), 0.2, 100, 1, 16, pool_opts=dict(S=8, L=3, K=16, seed=4))


def test_long_rows(fp):
    """Rows of thousands of edges (row tables of up to 2^11 entries)."""
    g = synth.chung_lu(6000, 90000, 2.05, 200, seed=2071)
    say(f"case: guide layout, long rows, max out-degree {g.degrees().max()}")
    check_all(fp, g, 0.15, 80, 19, 12, pool_opts=dict(S=24, L=3, K=32, seed=77))


def test_row_totals_above_32_bits(fp):
    g = synth.chung_lu(3000, 40000, 2.1, 2_000_000_000, seed=2072)
    say(f"case: guide layout, weights up to {g.w.max()}")
    check_all(fp, g, 0.15, 60, 5, 8, pool_opts=dict(S=16, L=2, K=8, seed=3), narrow_too=False)


def shaped_graph():
    """Rows whose thresholds crowd into a few entries: tiny edges between
    giants, doubling weights, one giant among ones, equal weights."""
    rng = np.random.default_rng(2090)
    n = 400
    rows = []
    big = 0xFFFFFFFF
    for u in range(n):
        kind = u % 8
        if kind == 0:
            w = np.r_[[big], np.ones(int(rng.integers(3, 900))), [big]]
        elif kind == 1:
            w = 2 ** (np.arange(int(rng.integers(2, 33))) % 32)
        elif kind == 2:
            d = int(rng.integers(2, 3000))
            w = np.ones(d)
            w[rng.integers(0, d)] = big
        elif kind == 3:
            w = np.ones(int(rng.integers(1, 70)))
        elif kind == 4:
            w = np.minimum(rng.zipf(1.1, int(rng.integers(1, 5000))), big)
        elif kind == 5:
            w = np.r_[np.ones(200), [big] * 3, np.ones(300), [big], np.ones(5)]
        elif kind == 6:
            w = np.zeros(0)  # no out-edges
        else:
            w = rng.integers(1, 1 << 32, int(rng.integers(1, 200)), dtype=np.uint64)
        rows.append(np.asarray(w, np.uint64))
    src = np.concatenate([np.full(r.size, u, np.uint32) for u, r in enumerate(rows)])
    dst = rng.integers(0, n, src.size).astype(np.uint32)
    w = np.concatenate(rows).astype(np.uint32)
    return synth.csr_from_edges(n, src, dst, w)


def test_crowded_thresholds(fp):
    g = shaped_graph()
    say(f"case: guide layout, crowded thresholds, m {g.m}")
    check_all(fp, g, 0.1, 300, 23, 10, pool_opts=dict(S=32, L=3, K=64, seed=9), narrow_too=False)


def long_crowded_graph():
    """Rows of more than 1024 edges (entries built a run of 16 at a time)
    whose light edges crowd many thresholds into few entries while holding
    a real share of the weight, so that walks do draw there: one heavy edge
    with three times the weight of thousands of unit edges, a 1-1-1-50
    pattern, Zipf(1.05) weights, unit weights just above 1024 edges; short
    rows and rows without out-edges between them."""
    rng = np.random.default_rng(2093)
    n = 320
    rows = []
    for u in range(n):
        kind = u % 6
        if kind == 0:
            d = int(rng.integers(1100, 4000))
            w = np.ones(d, np.uint64)
            w[int(rng.integers(0, d))] = 3 * (d - 1)
        elif kind == 1:
            d = int(rng.integers(1100, 4000))
            w = np.where(np.arange(d) % 4 == 3, 50, 1).astype(np.uint64)
        elif kind == 2:
            w = np.minimum(rng.zipf(1.05, int(rng.integers(2000, 6000))), 0xFFFFFFFF).astype(np.uint64)
        elif kind == 3:
            w = np.ones(int(rng.integers(1025, 1100)), np.uint64)
        elif kind == 4:
            w = rng.integers(1, 1000, int(rng.integers(1, 60))).astype(np.uint64)
        else:
            w = np.zeros(0, np.uint64)
        rows.append(w)
    src = np.concatenate([np.full(r.size, u, np.uint32) for u, r in enumerate(rows)])
    dst = rng.integers(0, n, src.size).astype(np.uint32)
    return synth.csr_from_edges(n, src, dst, np.concatenate(rows).astype(np.uint32))


def test_crowded_long_rows(fp):
    g = long_crowded_graph()
    say(f"case: guide layout, crowded long rows, m {g.m}, max out-degree {g.degrees().max()}")
    check_all(fp, g, 0.15, 400, 29, 16, pool_opts=dict(S=32, L=3, K=32, seed=11), narrow_too=False)


def test_borrowed_csr_rebuild(fp):
    """New weights written into a borrowed CSR, then a rebuild: the oracle's
    result for the new weights (or, when they need more child tables than
    the graph was made with, a failed check)."""
    import torch

    say("case: guide layout, borrowed CSR + rebuild")
    small = synth.small_graph()
    ro = torch.from_numpy(small.row_offsets.view(np.int64)).cuda()
    col = torch.from_numpy(small.col.view(np.int32)).cuda()
    w = torch.from_numpy(small.w.view(np.int32)).cuda()
    G = fp.Graph(n=small.n, row_offsets=ro, col=col, w=w, layout=fp.FPPR_LAYOUT_GUIDE)
    G.build_pool(S=8, L=3, K=16, alpha=0.2, seed=4)
    for k, w2 in enumerate([(small.w.astype(np.uint64) * 7 % 1000 + 1).astype(np.uint32), small.w.copy()]):
        w.copy_(torch.from_numpy(w2.view(np.int32)).cuda())
        G.rebuild()
        G.check()
        g2 = synth.CSRGraph(small.n, small.row_offsets, small.col, w2)
        og = O.Graph.from_csr(g2)
        pool = O.Pool(og, S=8, L=3, K=16, alpha=0.2, seed=4)
        assert np.array_equal(G.export_pool(), pool.entries())
        out = fp.run(G, 0.2, 50, 8 + k, topk=5, stitch=True, stats=True)
        ref = O.run(og, 0.2, 50, 8 + k, topk=5, pool=pool)
        compare(out, ref, 5)
        stats_equal(out, ref.stats)
    G.close()


def test_rebuild_beyond_room_fails_check(fp):
    """A graph created with equal weights has no child tables, so it gets
    room for its row tables plus the slack; new weights that crowd every
    row (one giant edge among 63 light ones: a child table of about 64
    entries per row, 4M in all) need more. The rebuild's check reports it
    (recreate the graph), and a graph created from the new weights gives the
    oracle's results."""
    import torch

    n, deg = 1 << 16, 64
    rng = np.random.default_rng(2101)
    src = np.repeat(np.arange(n, dtype=np.uint32), deg)
    dst = rng.integers(0, n, src.size).astype(np.uint32)
    g = synth.csr_from_edges(n, src, dst, np.ones(src.size, np.uint32))
    say(f"case: guide layout, rebuild beyond the created room, m {g.m}")
    ro = torch.from_numpy(g.row_offsets.view(np.int64)).cuda()
    col = torch.from_numpy(g.col.view(np.int32)).cuda()
    w = torch.from_numpy(g.w.view(np.int32)).cuda()
    G = fp.Graph(n=g.n, row_offsets=ro, col=col, w=w, layout=fp.FPPR_LAYOUT_GUIDE)
    G.check()
    w2 = np.ones(g.m, np.uint32)
    w2[g.row_offsets[:-1].astype(np.int64)] = 1 << 31  # the first edge of every row
    w.copy_(torch.from_numpy(w2.view(np.int32)).cuda())
    G.rebuild()
    with pytest.raises(fp.FpprError) as ei:
        G.check()
    assert "recreate" in str(ei.value)
    torch.cuda.synchronize()
    G.close()
    g2 = synth.CSRGraph(g.n, g.row_offsets, g.col, w2)
    G2 = fp.Graph(g2, layout=fp.FPPR_LAYOUT_GUIDE)
    sample = np.sort(rng.choice(n, 96, replace=False)).astype(np.uint32)
    out = fp.run(G2, 0.15, 40, 12, topk=8, sources=sample, stats=True)
    ref = O.run(O.Graph.from_csr(g2), 0.15, 40, 12, topk=8, sources=sample)
    compare(out, ref, 8)
    stats_equal(out, ref.stats)
    G2.close()


def test_source_lists_and_lane_keys(fp):
    """A source list with duplicates and nodes of every class, then a server
    (many descriptors on one graph: the per-lane-key form) whose every query
    equals its run alone and the oracle."""
    g = synth.chung_lu(5000, 60000, 2.2, 255, seed=2091)
    say("case: guide layout, source lists, server")
    G = fp.Graph(g, layout=fp.FPPR_LAYOUT_GUIDE)
    G.build_pool(S=16, L=3, K=32, alpha=0.15, seed=6)
    og = O.Graph.from_csr(g)
    pool = O.Pool(og, S=16, L=3, K=32, alpha=0.15, seed=6)
    rng = np.random.default_rng(2092)
    deg = g.degrees()
    src = np.r_[np.nonzero(deg == 0)[0][:5], np.nonzero((deg > 0) & (deg <= 16))[0][:5],
                np.argsort(deg)[-5:], rng.integers(0, g.n, 40), [7, 7, 7]].astype(np.uint32)
    for stitch in (False, True):
        out = fp.run(G, 0.15, 333, 12, sources=src, topk=20, stitch=stitch, stats=True)
        ref = O.run(og, 0.15, 333, 12, sources=src, topk=20, pool=pool if stitch else None)
        compare(out, ref, 20)
        stats_equal(out, ref.stats)
    S = fp.Server(G, mode="continuous", max_requests=8, slice_walks=1 << 16)
    qs = [dict(sources=rng.integers(0, g.n, int(rng.integers(1, 40))).astype(np.uint32),
               R=int(rng.choice([100, 1000, 3000])), seed=100 + i, topk=16, stitch=bool(i % 2)) for i in range(12)]
    ids = [S.submit(q["sources"], q["R"], 0.15, q["seed"], q["topk"], q["stitch"]) for q in qs]
    outs = [S.wait(i) for i in ids]
    S.close()
    for q, (topk, digest, _) in zip(qs, outs):
        ref = O.run(og, 0.15, q["R"], q["seed"], sources=q["sources"], topk=q["topk"],
                    pool=pool if q["stitch"] else None, want_counts=False)
        assert np.array_equal(topk, ref.topk) and np.array_equal(digest, ref.digest)
    G.close()


def test_medium_rmat_all_sources(fp):
    """R-MAT scale 20, every source: digests, distinct counts, top-k and
    statistics of all 2^20 sources against the oracle."""
    import torch

    say("case: guide layout, R-MAT scale 20, all sources")
    g = synth.medium_graph()
    G = fp.Graph(g, layout=fp.FPPR_LAYOUT_GUIDE)
    out = fp.run(G, 0.15, 200, 2, topk=32, counts=True, stats=True)
    og = O.Graph.from_csr(g)
    ref = O.run(og, 0.15, 200, 2, topk=32, want_counts=False)
    torch.cuda.synchronize()
    assert np.array_equal(u32(out.n_distinct), ref.n_distinct)
    assert np.array_equal(u32(out.topk), ref.topk)
    assert np.array_equal(u64(out.digest), ref.digest)
    stats_equal(out, ref.stats)
    G.close()


def test_scale24_stitched_sampled(fp):
    """R-MAT scale 24 with the pool (S=32, L=3, K=64): the whole pool and a
    stratified sample of 8192 sources (hubs, small, dangling, random)
    against the oracle, from a run over all 2^24 sources in the benchmark's
    launch configuration."""
    import torch

    say("case: guide layout, scale-24 generate")
    g = synth.scale24_graph()
    cfg = synth.SCALE24
    st = cfg["stitch"]
    say("case: guide layout, scale-24 GPU graph + pool")
    G = fp.Graph(g, layout=fp.FPPR_LAYOUT_GUIDE)
    G.build_pool(S=st["S"], L=st["L"], K=st["K"], alpha=cfg["alpha"], seed=st["seed"])
    say("case: guide layout, scale-24 GPU run, all sources")
    out = fp.run(G, cfg["alpha"], cfg["R"], cfg["seed"], topk=cfg["topk"], stitch=True, counts=False, stats=True)
    torch.cuda.synchronize()
    say("case: guide layout, scale-24 oracle pool")
    og = O.Graph.from_csr(g)
    pool = O.Pool(og, S=st["S"], L=st["L"], K=st["K"], alpha=cfg["alpha"], seed=st["seed"])
    assert np.array_equal(G.export_pool(), pool.entries())
    sample = synth.stratified_sources(g, 8192, seed=12, hub_threshold=cfg["hub_threshold"], small_max=st["S"])
    say("case: guide layout, scale-24 oracle sample")
    ref = O.run(og, cfg["alpha"], cfg["R"], cfg["seed"], sources=sample, topk=cfg["topk"], pool=pool)
    compare(out, ref, cfg["topk"], counts=False, sample=sample)
    out_s = fp.run(G, cfg["alpha"], cfg["R"], cfg["seed"], sources=sample, topk=cfg["topk"], stitch=True)
    compare(out_s, ref, cfg["topk"])
    stats_equal(out_s, ref.stats)
    assert out.stats_dict()["walks"] == g.n * cfg["R"]
    G.close()


def test_batch_capture_and_mixed_layouts(fp):
    """Guide-table graphs in one batch (plain and stitched, all nodes and a
    source list): every item equals its plain run and the oracle, captured
    replays equal the eager run; a batch that mixes guide tables with the
    tree layouts is refused at creation."""
    import torch

    say("case: guide layout, batch + capture")
    specs = [(synth.chung_lu(3000, 30000, 2.1, 255, seed=2101), 0.1, 64, 11, 8, None, False),
             (synth.chung_lu(500, 4000, 2.5, 255, seed=2102), 0.2, 256, 12, 16, None, True),
             (synth.chung_lu(8000, 120000, 2.2, 255, seed=2103), 0.15, 64, 13, 32,
              np.arange(0, 8000, 5, dtype=np.uint32), True)]
    items = []
    for g, alpha, R, seed, k, src, stitch in specs:
        G = fp.Graph(g, layout=fp.FPPR_LAYOUT_GUIDE)
        if stitch:
            G.build_pool(S=16, L=3, K=32, alpha=alpha, seed=seed + 100)
        items.append(dict(csr=g, graph=G, alpha=alpha, R=R, seed=seed, topk=k, sources=src, stitch=stitch))
    B = fp.Batch(items, rebuild=True)
    B.run()
    B.check()
    torch.cuda.synchronize()
    want = []
    for it, ob in zip(items, B.outputs):
        og = O.Graph.from_csr(it["csr"])
        pool = O.Pool(og, S=16, L=3, K=32, alpha=it["alpha"], seed=it["seed"] + 100) if it["stitch"] else None
        ref = O.run(og, it["alpha"], it["R"], it["seed"], sources=it["sources"], topk=it["topk"], pool=pool)
        assert np.array_equal(u32(ob.counts), ref.counts)
        assert np.array_equal(u32(ob.topk), ref.topk)
        assert np.array_equal(u64(ob.digest), ref.digest)
        want.append((u32(ob.counts).copy(), u64(ob.digest).copy()))
    stream = torch.cuda.Stream()
    B.capture(stream)
    for rep in range(2):
        for o in B.outputs:
            o.counts.fill_(-1)
            o.digest.fill_(-1)
        torch.cuda.synchronize()
        B.launch(stream)
        stream.synchronize()
        for (c, d), o in zip(want, B.outputs):
            assert np.array_equal(u32(o.counts), c) and np.array_equal(u64(o.digest), d), rep
    B.close()
    Gn = fp.Graph(specs[0][0], layout=fp.FPPR_LAYOUT_NARROW)
    mixed = [dict(items[0]), dict(items[0], graph=Gn)]
    with pytest.raises(fp.FpprError):
        fp.Batch(mixed)
    Gn.close()
    for it in items:
        it["graph"].close()


def test_static_entry_and_autotune(fp):
    """The entry point that allocates nothing gives fppr_run's results on a
    guide graph; the autotuner (whose hub thresholds mean nothing here)
    leaves a configuration whose run equals the oracle."""
    import torch

    say("case: guide layout, static entry + autotune")
    g = synth.chung_lu(20000, 240000, 2.2, 255, seed=2111)
    G = fp.Graph(g, layout=fp.FPPR_LAYOUT_GUIDE)
    p = fp.make_params(0.15, 64, 41, 8, False, True, True, True)
    out_s = fp.alloc_outputs(g.n, 64, 8, True, True, True)
    fp.fppr_run_static(G, p, None, g.n, out_s)
    ref_run = fp.run(G, 0.15, 64, 41, topk=8)
    torch.cuda.synchronize()
    assert np.array_equal(u32(out_s.counts), u32(ref_run.counts))
    assert np.array_equal(u64(out_s.digest), u64(ref_run.digest))
    pools = [dict(S=16, L=2, K=32, seed=31), dict(S=32, L=3, K=64, seed=32)]
    r = G.autotune(0.15, 64, 41, hub_thresholds=[0], blocks_per_cu=[0, 2], pools=pools, sample=4096, reps=1)
    stitch = r["pool"] >= 0
    o = fp.run(G, 0.15, 64, 41, topk=8, stitch=stitch, blocks_per_cu=r["blocks_per_cu"])
    torch.cuda.synchronize()
    og = O.Graph.from_csr(g)
    pool = None
    if stitch:
        po = pools[r["pool"]]
        pool = O.Pool(og, S=po["S"], L=po["L"], K=po["K"], alpha=0.15, seed=po["seed"])
    ref = O.run(og, 0.15, 64, 41, topk=8, pool=pool)
    assert np.array_equal(u32(o.counts), ref.counts)
    assert np.array_equal(u64(o.digest), ref.digest)
    G.close()
