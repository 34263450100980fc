"""The two graph layouts (64-bit prefixes, and 32-bit prefixes for graphs whose
row totals fit in 32 bits) give bit-identical results, against each other and
against the oracle; the narrow layout is refused where it does not fit and
chosen by default where it does; a rebuild that breaks a narrow graph's
32-bit bound is reported."""
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
    fppr.lib()
    return fppr


def same(a, b):
    import torch

    torch.cuda.synchronize()
    for name in ("topk", "counts", "n_distinct", "digest", "stats"):
        x, y = getattr(a, name), getattr(b, name)
        assert (x is None) == (y is None), name
        if x is not None:
            assert torch.equal(x, y), name


@pytest.mark.parametrize("H", [8, 40, UINT32_MAX])
def test_narrow_equals_wide_and_oracle(fp, H):
    """A Chung-Lu graph with rows of up to thousands of edges (trees of
    several levels in both layouts): every source, plain and stitched."""
    g = synth.chung_lu(6000, 90000, 2.05, 200, seed=2071)
    say(f"case: layouts, hub threshold {H}, max out-degree {g.degrees().max()}")
    Gn = fp.Graph(g, hub_threshold=H, layout=fp.FPPR_LAYOUT_NARROW)
    Gw = fp.Graph(g, hub_threshold=H, layout=fp.FPPR_LAYOUT_WIDE)
    assert Gn.layout() == fp.FPPR_LAYOUT_NARROW and Gw.layout() == fp.FPPR_LAYOUT_WIDE
    og = O.Graph.from_csr(g)
    for stitch in (False, True):
        pool = None
        if stitch:
            for G in (Gn, Gw):
                G.build_pool(S=24, L=3, K=32, alpha=0.15, seed=77)
            assert np.array_equal(Gn.export_pool(), Gw.export_pool())
            pool = O.Pool(og, S=24, L=3, K=32, alpha=0.15, seed=77)
            assert np.array_equal(Gn.export_pool(), pool.entries())
        kw = dict(topk=12, stitch=stitch, counts=True, digests=True, stats=True)
        a = fp.run(Gn, 0.15, 80, 19, **kw)
        b = fp.run(Gw, 0.15, 80, 19, **kw)
        same(a, b)
        ref = O.run(og, 0.15, 80, 19, topk=12, pool=pool)
        assert np.array_equal(a.counts.cpu().numpy().view(np.uint32), ref.counts)
        assert np.array_equal(a.topk.cpu().numpy().view(np.uint32), ref.topk)
        st = a.stats_dict()
        for key in ("walks", "moves", "steps", "plain_moves", "stitched_moves", "probe_log_sum"):
            assert st[key] == ref.stats[key], key


def test_large_weights_select_wide(fp):
    """Weights near 2^31: row totals exceed 32 bits, the graph is wide, and
    the results still match the oracle."""
    g = synth.chung_lu(3000, 40000, 2.1, 2_000_000_000, seed=2072)
    say(f"case: large weights, max weight {g.w.max()}")
    with pytest.raises(fp.FpprError):
        fp.Graph(g, layout=fp.FPPR_LAYOUT_NARROW)
    G = fp.Graph(g)
    assert G.layout() == fp.FPPR_LAYOUT_WIDE
    src = np.arange(0, g.n, 7, dtype=np.uint32)
    out = fp.run(G, 0.2, 64, 23, sources=src, topk=8)
    ref = O.run(O.Graph.from_csr(g), 0.2, 64, 23, sources=src, topk=8)
    import torch

    torch.cuda.synchronize()
    assert np.array_equal(out.counts.cpu().numpy().view(np.uint32), ref.counts)
    assert np.array_equal(out.topk.cpu().numpy().view(np.uint32), ref.topk)


def test_rebuild_past_the_narrow_bound_is_reported(fp):
    """A narrow graph over borrowed device arrays whose weights are rewritten
    so that a row total passes 2^32 - 1: the rebuild's check fails."""
    import torch

    g = synth.chung_lu(2000, 20000, 2.1, 100, seed=2073)
    say("case: narrow graph, rebuild with huge weights")
    ro = torch.from_numpy(g.row_offsets.view(np.int64)).cuda()
    col = torch.from_numpy(g.col.view(np.int32)).cuda()
    w = torch.from_numpy(g.w.view(np.int32)).cuda()
    G = fp.Graph(n=g.n, row_offsets=ro, col=col, w=w, layout=fp.FPPR_LAYOUT_NARROW)
    assert fp.Graph(g).layout() == fp.FPPR_LAYOUT_NARROW  # narrow by default where it fits
    assert G.layout() == fp.FPPR_LAYOUT_NARROW
    big = np.full(g.m, 0x7FFFFFFF, dtype=np.uint32)
    w.copy_(torch.from_numpy(big.view(np.int32)).cuda())
    G.rebuild()
    with pytest.raises(fp.FpprError) as ei:
        G.check()
    assert "32 bits" in str(ei.value) or "2^32" in str(ei.value)
    torch.cuda.synchronize()


def test_narrow_threshold_changes_keep_results(fp):
    """Changing the hub threshold of a narrow graph (rows re-laid out, pool
    rebuilt) never changes results; they stay equal to a wide graph's."""
    g = synth.chung_lu(6000, 90000, 2.05, 200, seed=2074)
    say("case: narrow graph, hub threshold changes")
    G = fp.Graph(g, layout=fp.FPPR_LAYOUT_NARROW)
    Gw = fp.Graph(g, layout=fp.FPPR_LAYOUT_WIDE)
    for X in (G, Gw):
        X.build_pool(S=16, L=2, K=16, alpha=0.2, seed=9)
    kw = dict(topk=10, stitch=True, counts=True, digests=True, stats=True)
    ref = fp.run(Gw, 0.2, 48, 31, **kw)
    for H in (8, 100, 3000, UINT32_MAX, 8):
        G.set_hub_threshold(H)
        G.rebuild()
        G.check()
        same(fp.run(G, 0.2, 48, 31, **kw), ref)
