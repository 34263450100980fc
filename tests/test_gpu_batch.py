"""Batches through the C-ABI: one persistent walk launch over several graphs
and source sets gives every item exactly its plain-run (and oracle) result;
a captured HIP graph replays to the same results."""
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


@pytest.fixture(scope="module")
def items(fp):
    """Six items of uneven size: different graphs, alphas, walk budgets,
    source subsets, plain and stitched, both layouts in one table."""
    specs = [
        (synth.chung_lu(3000, 30000, 2.1, 255, seed=2001), 0.1, 64, 11, 8, None, False),
        (synth.chung_lu(500, 4000, 2.5, 255, seed=2002), 0.2, 256, 12, 16, None, True),
        (synth.chung_lu(20000, 300000, 2.3, 255, seed=2003), 0.15, 64, 13, 32,
         np.arange(0, 20000, 7, dtype=np.uint32), False),
        (synth.small_graph(), 0.2, 100, 1, 16, None, False),
        (synth.chung_lu(1000, 9000, 2.2, 255, seed=2004), 0.15, 33, 14, 5,
         np.array([3, 999, 3, 0, 500], dtype=np.uint32), True),
        (synth.chung_lu(64, 300, 2.1, 255, seed=2005), 0.1, 256, 15, 64, None, False),
    ]
    out = []
    for i, (g, alpha, R, seed, k, src, stitch) in enumerate(specs):
        G = fp.Graph(g, layout=fp.FPPR_LAYOUT_NARROW if i % 2 == 0 else fp.FPPR_LAYOUT_WIDE)
        if stitch:
            G.build_pool(S=16, L=3, K=32, alpha=alpha, seed=seed + 100)
        out.append(dict(csr=g, graph=G, alpha=alpha, R=R, seed=seed, topk=k, sources=src,
                        stitch=stitch))
    return out


def test_batch_equals_plain_and_oracle(fp, items):
    import torch

    say("case: batch of 6 items vs plain runs and the oracle")
    B = fp.Batch(items)
    B.run()
    B.check()
    total_walks = 0
    for it, ob in zip(items, B.outputs):
        op = fp.run(it["graph"], it["alpha"], it["R"], it["seed"], sources=it["sources"],
                    topk=it["topk"], stitch=it["stitch"])
        torch.cuda.synchronize()
        for name in ("counts", "n_distinct", "topk"):
            assert np.array_equal(u32(getattr(ob, name)), u32(getattr(op, name))), name
        assert np.array_equal(u64(ob.digest), u64(op.digest))
        og = O.Graph.from_csr(it["csr"])
        pool = None
        if it["stitch"]:
            pool = O.Pool(og, S=16, L=3, K=32, alpha=it["alpha"], seed=it["seed"] + 100)
        ref = O.run(og, it["alpha"], it["R"], it["seed"], sources=it["sources"], topk=it["topk"],
                    pool=pool)
        assert np.array_equal(u32(ob.counts), ref.counts)
        assert np.array_equal(u32(ob.topk), ref.topk)
        assert np.array_equal(u64(ob.digest), ref.digest)
        total_walks += ref.stats["walks"]
    assert B.stats_dict()["walks"] == total_walks
    B.close()


def test_batch_capture_replays_match_eager(fp, items):
    """The captured graph is replayed several times with eager work and
    synchronisations between replays; every replay reproduces the eager
    results (outputs are overwritten with junk before each replay)."""
    import torch

    say("case: batch capture + replays")
    B = fp.Batch(items)
    B.run()
    torch.cuda.synchronize()
    want = [(u32(o.counts).copy(), u32(o.topk).copy(), u64(o.digest).copy()) for o in B.outputs]
    stream = torch.cuda.Stream()
    B.capture(stream)
    for rep in range(3):
        for o in B.outputs:
            o.counts.fill_(-1)
            o.topk.fill_(-1)
            o.digest.fill_(-1)
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        B.launch(stream)
        stream.synchronize()
        for (c, t, d), o in zip(want, B.outputs):
            assert np.array_equal(u32(o.counts), c), rep
            assert np.array_equal(u32(o.topk), t), rep
            assert np.array_equal(u64(o.digest), d), rep
        del junk
    B.close()


def test_batch_workload_smallest_graphs_vs_oracle(fp):
    """The 64-graph batch workload: the 8 smallest graphs in one batch, each
    checked against the oracle."""
    import torch

    say("case: batch workload, 8 smallest graphs")
    specs = sorted(synth.batch_specs(), key=lambda s: s["n"])[:8]
    its = []
    for sp in specs:
        g = synth.batch_graph(sp)
        its.append(dict(csr=g, graph=fp.Graph(g), alpha=sp["alpha"], R=sp["R"],
                        seed=sp["walk_seed"], topk=16, sources=None, stitch=False))
    B = fp.Batch(its, counts=False)
    B.run()
    torch.cuda.synchronize()
    for it, o in zip(its, B.outputs):
        ref = O.run(O.Graph.from_csr(it["csr"]), it["alpha"], it["R"], it["seed"], topk=16,
                    want_counts=False)
        assert np.array_equal(u32(o.topk), ref.topk)
        assert np.array_equal(u64(o.digest), ref.digest)
    B.close()


def test_relayout_and_launch_width_never_change_results(fp):
    """fppr_graph_set_hub_threshold (trees on/off, pool rebuilt) and the
    walk-launch width leave every result bit-identical."""
    import torch

    say("case: re-layout + launch width invariance")
    g = synth.chung_lu(5000, 80000, 2.1, 255, seed=2010)
    G = fp.Graph(g)
    G.build_pool(S=16, L=3, K=32, alpha=0.15, seed=9)
    base = fp.run(G, 0.15, 64, 21, topk=8, stitch=True)
    want = (u32(base.counts), u64(base.digest), u32(base.topk))
    for H, bpc in ((0xFFFFFFFF, 0), (64, 1), (8, 2), (8, 3)):
        G.set_hub_threshold(H)
        o = fp.run(G, 0.15, 64, 21, topk=8, stitch=True, blocks_per_cu=bpc)
        torch.cuda.synchronize()
        assert np.array_equal(u32(o.counts), want[0]), (H, bpc)
        assert np.array_equal(u64(o.digest), want[1]), (H, bpc)
        assert np.array_equal(u32(o.topk), want[2]), (H, bpc)
    info = G.info()
    assert info["hubs"] == int((g.degrees() > 8).sum())


def test_autotune_choice_matches_oracle(fp):
    """The tuner leaves the graph in its chosen configuration; a run in that
    configuration equals the oracle given the same pool parameters."""
    import torch

    say("case: autotune")
    g = synth.chung_lu(20000, 240000, 2.2, 255, seed=2011)
    G = fp.Graph(g)
    pools = [dict(S=16, L=2, K=32, seed=31), dict(S=32, L=3, K=64, seed=32)]
    r = G.autotune(0.15, 64, 41, hub_thresholds=[8, 64, 0xFFFFFFFF], blocks_per_cu=[0, 2],
                   pools=pools, sample=4096, reps=2)
    say(f"  tuned: {r}")
    assert r["hub_threshold"] in (8, 64, 0xFFFFFFFF)
    assert r["blocks_per_cu"] in (0, 2)
    assert r["pool"] in (-1, 0, 1)
    assert r["trials"] == 3 + 1 + len(pools)
    stitch = r["pool"] >= 0
    assert (G.info()["small"] > 0) == stitch
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
    # forcing the other choice still works: plain walks on a graph without a pool
    G.set_hub_threshold(8)
    o2 = fp.run(G, 0.15, 64, 41, topk=8, stitch=False)
    ref2 = O.run(og, 0.15, 64, 41, topk=8)
    assert np.array_equal(u64(o2.digest), ref2.digest)


def test_batch_with_rebuild_captured(fp, items):
    """FPPR_BATCH_REBUILD puts every graph's rebuild (prefixes, records,
    trees, pools) in front of the walks; captured and replayed it gives the
    eager results, and the launch width does not matter."""
    import torch

    say("case: batch with rebuild, captured, narrow launch")
    B0 = fp.Batch(items)
    B0.run()
    torch.cuda.synchronize()
    want = [(u32(o.counts).copy(), u64(o.digest).copy()) for o in B0.outputs]
    B0.close()
    B = fp.Batch(items, rebuild=True, blocks_per_cu=1)
    stream = torch.cuda.Stream()
    B.capture(stream)
    for rep in range(2):
        for o in B.outputs:
            o.counts.fill_(-1)
            o.digest.fill_(-1)
        torch.cuda.synchronize()
        B.launch(stream)
        B.check(stream)
        for (c, d), o in zip(want, B.outputs):
            assert np.array_equal(u32(o.counts), c), rep
            assert np.array_equal(u64(o.digest), d), rep
    B.close()


def test_destroy_waits_for_the_last_replay(fp, items):
    """fppr_batch_destroy right after a replay (no synchronisation by the
    caller) returns only once the replay has finished: the outputs read after
    it are complete, and the workspace can be freed at once."""
    import torch

    say("case: destroy right after an unsynchronised replay")
    B = fp.Batch(items)
    B.run()
    torch.cuda.synchronize()
    want = [(u32(o.counts).copy(), u64(o.digest).copy()) for o in B.outputs]
    stream = torch.cuda.Stream()
    B.capture(stream)
    for o in B.outputs:
        o.counts.fill_(-1)
        o.digest.fill_(-1)
    torch.cuda.synchronize()
    B.launch(stream)
    outs = B.outputs
    B.close()
    B.workspace = None
    for (c, d), o in zip(want, outs):
        assert np.array_equal(u32(o.counts), c)
        assert np.array_equal(u64(o.digest), d)


def test_manifest_records_each_items_knobs(fp, items):
    """fppr_batch_manifest: every item's graph layout, hub threshold and pool
    (S, L, K, seed), its parameters, and a walk table that tiles the launch."""
    say("case: batch manifest")
    B = fp.Batch(items, blocks_per_cu=2)
    m = B.manifest()
    assert m["launch_blocks_per_cu"] == 2 and len(m["items"]) == len(items)
    runs = []
    for it, mi in zip(items, m["items"]):
        assert mi["R"] == it["R"] and mi["seed"] == it["seed"] and mi["topk"] == it["topk"]
        assert abs(mi["alpha"] - it["alpha"]) < 1e-15 and mi["stitch"] == it["stitch"]
        assert mi["graph"]["n"] == it["csr"].n and mi["graph"]["m"] == it["csr"].m
        assert mi["graph"]["layout"] == ("narrow" if it["graph"].layout() == fp.FPPR_LAYOUT_NARROW else "wide")
        if it["stitch"]:
            assert mi["graph"]["pool"] == dict(S=16, L=3, K=32, seed=it["seed"] + 100, alpha=it["alpha"],
                                               small_nodes=it["graph"].info()["small"])
        n_src = it["csr"].n if it["sources"] is None else len(it["sources"])
        assert mi["sources"] == n_src and mi["all_nodes"] == (it["sources"] is None)
        if mi["launch_walks"]:
            runs.append((mi["first_walk_id"], mi["launch_walks"]))
    runs.sort()
    pos = 0
    for first, walks in runs:
        assert first == pos
        pos = first + (walks + 255) // 256 * 256
    assert pos == m["walk_ids"]
    B.close()
