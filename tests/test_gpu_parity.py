"""GPU path vs the CPU oracle, element by element, through the C-ABI.

Integer results, so the bar is bit-exact: sparse counts, distinct counts,
top-k lists, digests and the walk statistics.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu

UINT32_MAX = 0xFFFFFFFF


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fp():
    import torch

    from paper_1903_11749_amd import fppr

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    fppr.lib()  # fails loudly when the library is missing
    return fppr


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def u64(t):
    return t.cpu().numpy().view(np.uint64)


def compare(out, ref, R, k, counts=True, sample=None):
    """sample: row indices of `out` that correspond to ref's rows (None = all)."""
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


def graph_from_edges(n, edges, weights=None):
    src = np.array([e[0] for e in edges], dtype=np.uint32)
    dst = np.array([e[1] for e in edges], dtype=np.uint32)
    w = np.ones(len(edges), np.uint32) if weights is None else np.array(weights, np.uint64).astype(np.uint32)
    return synth.csr_from_edges(n, src, dst, w)


@pytest.fixture(scope="module")
def small():
    return synth.small_graph()


@pytest.mark.parametrize("layout", [0, 1, 2])
def test_small_plain_all_sources(fp, small, layout):
    """Chung-Lu n=2000, alpha=0.2, R=100, seed 1, top-16, every source; the
    default layout, wide and narrow."""
    say(f"case: small plain all sources, layout {layout}")
    G = fp.Graph(small, layout=layout)
    out = fp.run(G, 0.2, 100, 1, topk=16)
    ref = O.run(O.Graph.from_csr(small), 0.2, 100, 1, topk=16)
    compare(out, ref, 100, 16)
    stats_equal(out, ref.stats)


@pytest.mark.parametrize("layout", [1, 2])
@pytest.mark.parametrize("H", [2, 8, 9, 64, 100, 4096, UINT32_MAX])
def test_hub_threshold_is_results_invariant(fp, small, H, layout):
    """Rows above the threshold are searched through their prefix tree, the
    others by binary search: both pick the same edge as a flat search
    (integer form of Lemma 1), in either layout."""
    say(f"case: hub threshold H={H}, layout {layout}")
    G = fp.Graph(small, hub_threshold=H, layout=layout)
    info = G.info()
    deg = small.degrees()
    want = 0 if H == UINT32_MAX else int(np.count_nonzero(deg > max(H, 8)))
    assert info["hubs"] == want
    out = fp.run(G, 0.2, 100, 1, topk=16)
    ref = O.run(O.Graph.from_csr(small), 0.2, 100, 1, topk=16)
    compare(out, ref, 100, 16)
    stats_equal(out, ref.stats)


@pytest.mark.parametrize("layout", [1, 2])
@pytest.mark.parametrize("S,L,K,H", [(8, 3, 16, 4096), (32, 3, 64, 64), (4, 1, 1, 2), (64, 5, 8, 16),
                                     (16, 2, 32, UINT32_MAX)])
def test_small_stitched_and_pool(fp, small, S, L, K, H, layout):
    say(f"case: stitched S={S} L={L} K={K} H={H}, layout {layout}")
    alpha = 0.2
    G = fp.Graph(small, hub_threshold=H, layout=layout)
    G.build_pool(S=S, L=L, K=K, alpha=alpha, seed=99)
    og = O.Graph.from_csr(small)
    pool = O.Pool(og, S=S, L=L, K=K, alpha=alpha, seed=99)
    assert np.array_equal(G.export_pool(), pool.entries())
    out = fp.run(G, alpha, 100, 3, topk=16, stitch=True)
    ref = O.run(og, alpha, 100, 3, topk=16, pool=pool)
    compare(out, ref, 100, 16)
    stats_equal(out, ref.stats)


def test_sources_subset_ragged_and_duplicates(fp, small):
    """A ragged source list (duplicates, unsorted, 37 rows) gives each source
    exactly its all-sources result (I7)."""
    say("case: ragged source subset")
    G = fp.Graph(small)
    src = np.array([5, 1999, 17, 17, 0, 1234, 5] + list(range(100, 130)), dtype=np.uint32)
    out = fp.run(G, 0.2, 33, 12, sources=src, topk=7)
    ref = O.run(O.Graph.from_csr(small), 0.2, 33, 12, sources=src, topk=7)
    compare(out, ref, 33, 7)
    stats_equal(out, ref.stats)


@pytest.mark.parametrize("R,k", [(1, 1), (16, 16), (17, 3), (255, 0), (4096, 64)])
def test_walk_budget_edges(fp, small, R, k):
    say(f"case: R={R} k={k}")
    G = fp.Graph(small)
    src = np.arange(0, 2000, 97, dtype=np.uint32)
    out = fp.run(G, 0.15, R, 77, sources=src, topk=k)
    ref = O.run(O.Graph.from_csr(small), 0.15, R, 77, sources=src, topk=k)
    compare(out, ref, R, k)
    stats_equal(out, ref.stats)


def test_degenerate_graphs(fp):
    """Single dangling node; no edges; self-loops only; max weights; a walk
    that hits the move cap."""
    cases = [
        ("single node", graph_from_edges(1, []), 0.3),
        ("no edges", graph_from_edges(5, []), 0.3),
        ("self loops", graph_from_edges(3, [(0, 0), (1, 1), (2, 2), (2, 2)]), 0.3),
        ("max weights", graph_from_edges(4, [(0, 1), (0, 2), (0, 3), (1, 0), (2, 0)],
                                         [UINT32_MAX] * 5), 0.3),
        ("move cap", graph_from_edges(3, [(0, 1), (1, 2), (2, 0)]), 1e-12),
    ]
    for name, g, alpha in cases:
        say(f"case: degenerate {name}")
        G = fp.Graph(g)
        R = 4 if name == "move cap" else 50
        out = fp.run(G, alpha, R, 5, topk=min(3, R))
        ref = O.run(O.Graph.from_csr(g), alpha, R, 5, topk=min(3, R))
        compare(out, ref, R, min(3, R))
        stats_equal(out, ref.stats)


def test_empty_source_list_is_noop(fp, small):
    import torch

    say("case: empty source list")
    G = fp.Graph(small)
    p = fp.make_params(0.2, 10, 1, 2)
    ws = torch.zeros(64, dtype=torch.int64, device="cuda")
    out = fp.alloc_outputs(1, 10, 2)
    fp.fppr_run(G, p, torch.zeros(1, dtype=torch.int32, device="cuda"), 0, ws, out)
    torch.cuda.synchronize()


def test_invalid_arguments(fp, small):
    import torch

    say("case: invalid arguments")
    bad = [
        (small.n, small.row_offsets, np.where(np.arange(small.m) == 5, small.n, small.col), small.w),
        (small.n, small.row_offsets, small.col, np.where(np.arange(small.m) == 9, 0, small.w)),
    ]
    ro = small.row_offsets.copy()
    ro[10], ro[11] = ro[11] + 1, ro[10]
    bad.append((small.n, ro, small.col, small.w))
    for n, r, c, w in bad:
        with pytest.raises(fp.FpprError) as ei:
            fp.Graph(n=n, row_offsets=r, col=c.astype(np.uint32), w=w.astype(np.uint32))
        assert ei.value.status == fp.FPPR_INVALID_ARGUMENT
    G = fp.Graph(small)
    for kw in (dict(alpha=0.0, R=10), dict(alpha=1.0, R=10), dict(alpha=0.2, R=0),
               dict(alpha=0.2, R=10, topk=11)):
        with pytest.raises(fp.FpprError):
            fp.run(G, kw["alpha"], kw["R"], 1, sources=[1, 2], topk=kw.get("topk", 0))
    with pytest.raises(fp.FpprError):  # stitched without a pool
        fp.run(G, 0.2, 10, 1, sources=[1], stitch=True)
    G.build_pool(S=8, L=3, K=16, alpha=0.2, seed=1)
    with pytest.raises(fp.FpprError):  # pool built for another alpha
        fp.run(G, 0.3, 10, 1, sources=[1], stitch=True)
    with pytest.raises(fp.FpprError):  # source id out of range is reported
        fp.run(G, 0.2, 10, 1, sources=[1, small.n + 5])
    torch.cuda.synchronize()


def test_borrowed_device_csr_and_rebuild(fp, small):
    """A CSR already in HBM is borrowed; rebuilding after rewriting the
    weights in place gives the oracle's result for the new weights."""
    import torch

    say("case: borrowed CSR + rebuild")
    ro = torch.from_numpy(small.row_offsets.view(np.int64)).cuda()
    col = torch.from_numpy(small.col.view(np.int32)).cuda()
    w = torch.from_numpy(small.w.view(np.int32)).cuda()
    G = fp.Graph(n=small.n, row_offsets=ro, col=col, w=w)
    G.build_pool(S=8, L=3, K=16, alpha=0.2, seed=4)
    w2 = (small.w.astype(np.uint64) * 7 % 1000 + 1).astype(np.uint32)
    w.copy_(torch.from_numpy(w2.view(np.int32)).cuda())
    G.rebuild()
    G.check()
    g2 = synth.CSRGraph(small.n, small.row_offsets, small.col, w2)
    og = O.Graph.from_csr(g2)
    pool = O.Pool(og, S=8, L=3, K=16, alpha=0.2, seed=4)
    assert np.array_equal(G.export_pool(), pool.entries())
    out = fp.run(G, 0.2, 50, 8, topk=5, stitch=True)
    ref = O.run(og, 0.2, 50, 8, topk=5, pool=pool)
    compare(out, ref, 50, 5)


def test_medium_rmat_all_sources(fp):
    """R-MAT scale 20, alpha=0.15, R=200, top-32, every source: digests,
    distinct counts, top-k and statistics for all 2^20 sources; full counts
    for a sample."""
    say("case: medium R-MAT scale 20, all sources")
    g = synth.medium_graph()
    G = fp.Graph(g)
    out = fp.run(G, 0.15, 200, 2, topk=32, counts=True)
    og = O.Graph.from_csr(g)
    ref = O.run(og, 0.15, 200, 2, topk=32, want_counts=False)
    import torch

    torch.cuda.synchronize()
    assert np.array_equal(u32(out.n_distinct), ref.n_distinct)
    assert np.array_equal(u32(out.topk), ref.topk)
    assert np.array_equal(u64(out.digest), ref.digest)
    stats_equal(out, ref.stats)
    sample = synth.stratified_sources(g, 2048, seed=11)
    ref_s = O.run(og, 0.15, 200, 2, sources=sample, topk=32)
    compare(out, ref_s, 200, 32, sample=sample)


def test_scale24_stitched_hubs_sampled(fp):
    """R-MAT scale 24 with hubs (> 4096 edges) and short walks (S=32, L=3,
    K=64): the whole pool and a stratified sample of 8192 sources (every
    class: hubs, small, dangling, random) against the oracle, from a run over
    all 2^24 sources in the benchmark's launch configuration."""
    import torch

    say("case: scale-24 generate")
    g = synth.scale24_graph()
    cfg = synth.SCALE24
    st = cfg["stitch"]
    say("case: scale-24 GPU graph + pool")
    G = fp.Graph(g, hub_threshold=cfg["hub_threshold"])
    G.build_pool(S=st["S"], L=st["L"], K=st["K"], alpha=cfg["alpha"], seed=st["seed"])
    say("case: scale-24 GPU run, all sources")
    out = fp.run(G, cfg["alpha"], cfg["R"], cfg["seed"], topk=cfg["topk"], stitch=True,
                 counts=False)
    torch.cuda.synchronize()
    say("case: scale-24 oracle pool")
    og = O.Graph.from_csr(g)
    pool = O.Pool(og, S=st["S"], L=st["L"], K=st["K"], alpha=cfg["alpha"], seed=st["seed"])
    assert np.array_equal(G.export_pool(), pool.entries())
    sample = synth.stratified_sources(g, 8192, seed=12, hub_threshold=cfg["hub_threshold"],
                                      small_max=st["S"])
    say("case: scale-24 oracle sample")
    ref = O.run(og, cfg["alpha"], cfg["R"], cfg["seed"], sources=sample, topk=cfg["topk"], pool=pool)
    compare(out, ref, cfg["R"], cfg["topk"], counts=False, sample=sample)
    # the same sources run alone give the same counts (I7) and match in full
    out_s = fp.run(G, cfg["alpha"], cfg["R"], cfg["seed"], sources=sample, topk=cfg["topk"],
                   stitch=True)
    compare(out_s, ref, cfg["R"], cfg["topk"])
    stats_equal(out_s, ref.stats)
    st_all = out.stats_dict()
    assert st_all["walks"] == g.n * cfg["R"]
