"""Memory-bounded runs: with a workspace below fppr_plan the sources run in
blocks (one walk and one counting launch each); the results are identical to
the single-launch run, bit for bit, because walk keys do not depend on the
blocking."""
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


@pytest.fixture(scope="module")
def graph(fp):
    g = synth.chung_lu(20000, 220000, 2.2, 255, seed=2040)
    G = fp.Graph(g)
    G.build_pool(S=32, L=3, K=64, alpha=0.15, seed=41)
    return g, G


def same(a, b):
    import torch

    torch.cuda.synchronize()
    for name in ("topk", "counts", "n_distinct", "digest", "stats"):
        x, y = getattr(a, name), getattr(b, name)
        assert (x is None) == (y is None), name
        if x is not None:
            assert torch.equal(x, y), name


@pytest.mark.parametrize("case", [
    dict(R=64, sources=None, counts=True, stitch=False, div=7),
    dict(R=128, sources=None, counts=False, stitch=True, div=5),
    dict(R=300, sources="dup", counts=False, stitch=False, div=9),
    dict(R=5000, sources="sample", counts=False, stitch=True, div=4),
])
def test_blocked_equals_single_launch(fp, graph, case):
    g, G = graph
    say(f"case: blocked run {case}")
    if case["sources"] is None:
        src = None
    elif case["sources"] == "dup":
        src = np.concatenate([np.arange(0, g.n, 3), np.arange(0, g.n, 5)]).astype(np.uint32)
    else:
        src = np.arange(0, g.n, 61, dtype=np.uint32)
    n_src = g.n if src is None else src.size
    kw = dict(topk=16, stitch=case["stitch"], counts=case["counts"], digests=True, stats=True)
    full = fp.run(G, 0.15, case["R"], 9, sources=src, **kw)
    p = fp.make_params(0.15, case["R"], 9, 16, case["stitch"], case["counts"], True, True)
    need = fp.fppr_plan(G, p, n_src)
    block, ws = fp.fppr_plan_block(G, p, n_src, need // case["div"])
    assert 1 <= block < n_src and ws <= need // case["div"]
    part = fp.run(G, 0.15, case["R"], 9, sources=src, max_workspace=need // case["div"], **kw)
    same(full, part)
    if case["R"] <= 300 and src is not None:
        pool = O.Pool(O.Graph.from_csr(g), S=32, L=3, K=64, alpha=0.15, seed=41) if case["stitch"] else None
        ref = O.run(O.Graph.from_csr(g), 0.15, case["R"], 9, sources=src, topk=16, pool=pool,
                    want_counts=False)
        assert np.array_equal(part.digest.cpu().numpy().view(np.uint64), ref.digest)


def test_blocked_invalid_source_and_tiny_budget(fp, graph):
    g, G = graph
    say("case: blocked run with an invalid source in a later block; budget below one source")
    src = np.arange(0, 3000, dtype=np.uint32)
    src[2500] = g.n  # invalid, in the last block
    p = fp.make_params(0.15, 64, 9, 8, False, False, True, False)
    need = fp.fppr_plan(G, p, src.size)
    with pytest.raises(fp.FpprError):
        fp.run(G, 0.15, 64, 9, sources=src, topk=8, counts=False, stats=False, max_workspace=need // 6)
    with pytest.raises(fp.FpprError):
        fp.fppr_plan_block(G, p, src.size, 100)


def test_split_run_equals_blocked_and_oracle(fp):
    """A graph where about half the nodes have no out-edges: the all-nodes run
    sends their walks to the coin-only kernel; it equals the blocked run (which
    keeps every walk in the walk kernel) and the oracle, counts and statistics
    included."""
    import torch

    say("case: all-nodes run with the coin-only kernel vs blocked run vs oracle")
    g = synth.rmat(13, 8, .57, .19, .19, 100, seed=2050, zipf_s=1.3)
    assert (g.degrees() == 0).mean() > 0.25
    G = fp.Graph(g)
    kw = dict(topk=8, counts=True, digests=True, stats=True)
    full = fp.run(G, 0.15, 96, 13, **kw)
    p = fp.make_params(0.15, 96, 13, 8, False, True, True, True)
    part = fp.run(G, 0.15, 96, 13, max_workspace=fp.fppr_plan(G, p, g.n) // 3, **kw)
    same(full, part)
    ref = O.run(O.Graph.from_csr(g), 0.15, 96, 13, topk=8)
    torch.cuda.synchronize()
    assert np.array_equal(full.counts.cpu().numpy().view(np.uint32), ref.counts)
    assert np.array_equal(full.topk.cpu().numpy().view(np.uint32), ref.topk)
    st = full.stats_dict()
    for key in ("walks", "moves", "steps", "capped", "dangling_moves", "plain_moves"):
        assert st[key] == ref.stats[key], key


def test_profile_splits_walk_and_coin_only_time(fp):
    """The stage timer reports the walk kernel and the time the coin-only
    kernel (beside it on the graph's side stream) adds after it; their sum is
    the walk time, and runs without the coin-only kernel report 0 for it."""
    import torch

    say("case: stage timer of a split all-nodes run and of a source-list run")
    g = synth.rmat(13, 8, .57, .19, .19, 100, seed=2050, zipf_s=1.3)
    G = fp.Graph(g)
    p = fp.make_params(0.15, 96, 13, 8, False, False, True, False)
    for src in (None, np.arange(0, g.n, 2, dtype=np.uint32)):
        n_src = g.n if src is None else src.size
        ws = torch.empty((fp.fppr_plan(G, p, n_src) + 7) // 8, dtype=torch.int64, device="cuda")
        out = fp.alloc_outputs(n_src, 96, 8, counts=False, digests=True, stats=False)
        prof = fp.Profile()
        out.profile = prof
        s = None if src is None else torch.from_numpy(src.view(np.int32)).cuda()
        fp.fppr_run(G, p, s, n_src, ws, out, None)
        walk, _ = prof.read()
        kern, coin = prof.read_walk()
        assert kern > 0 and coin >= 0
        assert abs(kern + coin - walk) < 1e-3 + 1e-3 * walk
        if src is not None:
            assert coin < 0.05
