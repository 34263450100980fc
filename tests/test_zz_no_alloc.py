"""fppr_run_static (the entry point that allocates nothing: its workspace is
the library's fixed device array) gives exactly fppr_run's results, on calls
in a row with shrinking inputs, on a run larger than the array (blocked
inside), and refuses what cannot fit."""
import sys

import numpy as np
import pytest

import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu

STATIC_BYTES = 64 << 20  # FPPR_STATIC_SCRATCH_BYTES


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


def static_run(fp, G, alpha, R, seed, sources, topk, stitch=False, counts=True):
    import torch

    if sources is None:
        src, n_src = None, G.n
    else:
        src = torch.from_numpy(np.asarray(sources, dtype=np.uint32).view(np.int32)).cuda()
        n_src = int(src.numel())
    p = fp.make_params(alpha, R, seed, topk, stitch, counts, True, True)
    out = fp.alloc_outputs(n_src, R, topk, counts, True, True)
    fp.fppr_run_static(G, p, src, n_src, out)
    torch.cuda.synchronize()
    return out


def same(a, b, counts=True):
    assert np.array_equal(u32(a.topk), u32(b.topk))
    assert np.array_equal(u64(a.digest), u64(b.digest))
    if counts:
        assert np.array_equal(u32(a.counts), u32(b.counts))
        assert np.array_equal(u32(a.n_distinct), u32(b.n_distinct))
    assert a.stats_dict() == b.stats_dict()


def test_static_equals_run_two_calls_shrinking(fp):
    import torch

    g = synth.chung_lu(3000, 30000, 2.1, 255, seed=2101)
    G = fp.Graph(g)
    G.build_pool(S=16, L=3, K=32, alpha=0.15, seed=77)
    say("case: static run, all 3000 nodes, R 64, stitched")
    a = static_run(fp, G, 0.15, 64, 5, None, 16, stitch=True)
    b = fp.run(G, 0.15, 64, 5, topk=16, stitch=True)
    torch.cuda.synchronize()
    same(a, b)
    say("case: static run again, 100 sources (smaller input), plain")
    src = np.arange(7, 3000, 29, dtype=np.uint32)[:100]
    a2 = static_run(fp, G, 0.15, 64, 6, src, 16)
    b2 = fp.run(G, 0.15, 64, 6, sources=src, topk=16)
    torch.cuda.synchronize()
    same(a2, b2)
    ref = O.run(O.Graph.from_csr(g), 0.15, 64, 6, sources=src, topk=16)
    assert np.array_equal(u32(a2.counts), ref.counts)
    assert np.array_equal(u64(a2.digest), ref.digest)
    G.close()


def test_static_larger_than_its_array_runs_blocked(fp):
    import torch

    g = synth.chung_lu(2000, 20000, 2.1, 255, seed=2102)
    G = fp.Graph(g)
    R = 20000
    src = np.arange(0, 2000, 2, dtype=np.uint32)  # 1000 sources: 80 MB of endpoints
    p = fp.make_params(0.2, R, 9, 32, False, False, True, True)
    assert fp.fppr_plan(G, p, src.size) > STATIC_BYTES
    say("case: static run above the array size (blocked), R 20000, 1000 sources")
    a = static_run(fp, G, 0.2, R, 9, src, 32, counts=False)
    b = fp.run(G, 0.2, R, 9, sources=src, topk=32, counts=False)
    torch.cuda.synchronize()
    same(a, b, counts=False)
    say("case: static run after it, 10 sources")
    a2 = static_run(fp, G, 0.2, 300, 10, src[:10], 8, counts=False)
    b2 = fp.run(G, 0.2, 300, 10, sources=src[:10], topk=8, counts=False)
    torch.cuda.synchronize()
    same(a2, b2, counts=False)
    G.close()


def test_static_refuses_what_cannot_fit(fp):
    import torch

    g = synth.chung_lu(2000, 20000, 2.1, 255, seed=2103)
    G = fp.Graph(g)
    R = 20000
    n_src = 2000
    say("case: static run refusing endpoints that exceed the array")
    p = fp.make_params(0.2, R, 9, 8, False, False, True, False)
    out = fp.alloc_outputs(n_src, R, 8, False, True, False, endpoints=True)
    with pytest.raises(fp.FpprError) as ei:
        fp.fppr_run_static(G, p, None, n_src, out)
    assert ei.value.status == fp.FPPR_INVALID_ARGUMENT
    assert "static workspace" in str(ei.value)
    torch.cuda.synchronize()
    G.close()
