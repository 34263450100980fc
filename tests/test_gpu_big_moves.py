"""Exact big-move tables built on the GPU (Sec. 4.2, Algorithm 4, with the
size cap; weights stored as inclusive prefixes) are bit-identical to the
oracle's 62-bit tables for every small node: several graphs, degree bounds S, stop-rule sizes d, caps and alphas,
including levels through nodes without out-edges; on the R-MAT scale-20
graph the build is timed and a sample of small nodes recomputed."""
import sys

import numpy as np
import pytest

import synth
from oracle import big_moves as BM
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


CASES = [
    ("chung-lu S=8 d=16 cap=64 a=0.15", lambda: synth.chung_lu(400, 1600, 2.3, 20, seed=78), 8, 16, 64, 0.15),
    ("chung-lu S=16 d=32 cap=256 a=0.3", lambda: synth.chung_lu(600, 3000, 2.1, 1000, seed=79), 16, 32, 256, 0.3),
    ("r-mat S=32 d=32 cap=128", lambda: synth.rmat(10, 8, .57, .19, .19, 10000, seed=7, zipf_s=1.2), 32, 32, 128, 0.15),
    ("chung-lu S=4 d=100 cap=1024 a=0.5", lambda: synth.chung_lu(300, 900, 2.5, 5, seed=80), 4, 100, 1024, 0.5),
    ("r-mat S=8 d=6 cap=16 a=0.85", lambda: synth.rmat(9, 4, .57, .19, .19, 100, seed=9, zipf_s=1.5), 8, 6, 16, 0.85),
    ("r-mat dead ends S=4 d=64 cap=40", lambda: synth.rmat(11, 2, .45, .25, .25, 50, seed=12, zipf_s=1.5), 4, 64, 40, 0.1),
]


def compare(fp, g, ent, wts, cnt, S, d, cap, alpha, nodes):
    T = fp.fppr_alpha_threshold(alpha)
    offs, oe, ow = BM.table(g.row_offsets, g.col, g.w, nodes, T, d, max_entries=cap)
    bad = []
    for r, v in enumerate(nodes):
        c = int(cnt[v])
        if not (np.array_equal(ent[v, :c], oe[offs[r]:offs[r + 1]])
                and np.array_equal(wts[v, :c], np.cumsum(ow[offs[r]:offs[r + 1]], dtype=np.uint64))):
            bad.append(int(v))
    return bad


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_big_moves_equal_oracle(fp, case):
    import torch

    name, make, S, d, cap, alpha = case
    g = make()
    say(f"case: big moves, {name}, n={g.n}, m={g.m}")
    G = fp.Graph(g, layout=fp.FPPR_LAYOUT_NARROW)
    for slots in (16384, 3):  # every node its own workspace slot, or a few slots reused
        ent, wts, cnt = G.big_moves(S, d, cap, alpha, slots=slots)
        torch.cuda.synchronize()
        ent = ent.cpu().numpy().view(np.uint64)
        wts = wts.cpu().numpy().view(np.uint64)
        cnt = cnt.cpu().numpy().view(np.uint32)
        deg = g.degrees()
        small = np.flatnonzero((deg >= 1) & (deg <= S))
        assert np.all(cnt[(deg == 0) | (deg > S)] == 0)
        assert np.all((cnt[small] >= 1) & (cnt[small] <= cap))
        assert compare(fp, g, ent, wts, cnt, S, d, cap, alpha, small) == []


def test_big_moves_refusals(fp):
    g = synth.chung_lu(300, 900, 2.5, 5, seed=80)
    say("case: big moves, refused arguments")
    Gw = fp.Graph(g, layout=fp.FPPR_LAYOUT_WIDE)
    with pytest.raises(fp.FpprError):
        Gw.big_moves(8, 16, 64, 0.15)
    G = fp.Graph(g, layout=fp.FPPR_LAYOUT_NARROW)
    for S, d, cap, alpha in ((8, 16, 15, 0.15), (0, 16, 64, 0.15), (8, 0, 64, 0.15), (8, 16, 64, 0.0),
                             (8, 16, 8192, 0.15)):
        with pytest.raises(fp.FpprError):
            G.big_moves(S, d, cap, alpha)


def test_big_moves_scale20(fp):
    import torch

    g = synth.medium_graph()
    S, d, cap, alpha = 32, 32, 64, 0.15
    say(f"case: big moves, R-MAT scale 20, S={S} d={d} cap={cap}")
    G = fp.Graph(g)
    G.big_moves(S, d, cap, alpha)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    ent, wts, cnt = G.big_moves(S, d, cap, alpha)
    t1.record()
    torch.cuda.synchronize()
    deg = g.degrees()
    small = np.flatnonzero((deg >= 1) & (deg <= S))
    c = cnt.cpu().numpy().view(np.uint32)
    say(f"  {small.size} small nodes, {int(c.sum())} entries in {t0.elapsed_time(t1):.2f} ms")
    sample = np.sort(np.random.default_rng(5).choice(small, 300, replace=False))
    ent = ent.cpu().numpy().view(np.uint64)
    wts = wts.cpu().numpy().view(np.uint64)
    assert compare(fp, g, ent, wts, c, S, d, cap, alpha, sample) == []


@pytest.mark.parametrize("case", CASES[:3] + CASES[4:], ids=[c[0] for c in CASES[:3] + CASES[4:]])
def test_paper_design_walks_equal_oracle(fp, case):
    """Walks with alias picks and one exact big move at each small node
    (fppr_run_big_moves) give the oracle's endpoints and steps bit for bit."""
    import torch

    name, make, S, d, cap, alpha = case
    g = make()
    say(f"case: big-move walks, {name}")
    G = fp.Graph(g, layout=fp.FPPR_LAYOUT_NARROW)
    P, al = G.alias_tables()
    sl = G.alias_slots(P, al)
    nd = G.alias_nodes()
    bm = G.big_moves(S, d, cap, alpha)
    src = np.concatenate([np.arange(0, g.n, 13), [g.n - 1, 0, 0, g.n]]).astype(np.uint32)
    ep, st = fp.run_big_moves(G, sl, bm, S, alpha, 16, 987654321, sources=src)
    torch.cuda.synchronize()
    ep = ep.cpu().numpy().view(np.uint32).reshape(len(src), 16)
    st = st.cpu().numpy().view(np.uint32).reshape(len(src), 16)
    assert np.all(ep[-1] == 0xFFFFFFFF) and np.all(st[-1] == 0)
    T = fp.fppr_alpha_threshold(alpha)
    ref_ep, ref_st = BM.run_with_alias(g.row_offsets, g.col, g.w, S, d, cap, T, 987654321, 16, src[:-1])
    assert np.array_equal(ep[:-1], ref_ep) and np.array_equal(st[:-1], ref_st)


def test_paper_design_walks_scale20(fp):
    """R-MAT scale 20, R = 16 from every node, S = d = 32, cap = 64: timed
    beside the alias walks without big moves, and 128 sampled sources
    recomputed by the oracle."""
    import torch

    g = synth.medium_graph()
    S, d, cap, alpha = 32, 32, 64, 0.15
    say("case: big-move walks, R-MAT scale 20, R = 16 from every node")
    G = fp.Graph(g)
    P, al = G.alias_tables()
    sl = G.alias_slots(P, al)
    nd = G.alias_nodes()
    bm = G.big_moves(S, d, cap, alpha)
    fp.run_big_moves(G, sl, bm, S, alpha, 16, 3)
    torch.cuda.synchronize()
    res = {}
    for label, call in (("big moves + alias", lambda: fp.run_big_moves(G, sl, bm, S, alpha, 16, 3)),
                        ("alias only", lambda: fp.run_alias(G, nd, sl, alpha, 16, 3))):
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        ep, st = call()
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1)
        steps = int(st.to(torch.int64).sum().item())
        say(f"  {label}: {steps} steps in {ms:.2f} ms: {steps / ms * 1e3:.3e} walk-steps/s")
        res[label] = (ep, st)
    ep, st = res["big moves + alias"]
    sample = np.sort(np.random.default_rng(6).choice(g.n, 128, replace=False))
    e = ep.cpu().numpy().view(np.uint32).reshape(g.n, 16)[sample]
    s_ = st.cpu().numpy().view(np.uint32).reshape(g.n, 16)[sample]
    ref_ep, ref_st = BM.run_with_alias(g.row_offsets, g.col, g.w, S, d, cap,
                                       fp.fppr_alpha_threshold(alpha), 3, 16, sample)
    assert np.array_equal(e, ref_ep) and np.array_equal(s_, ref_st)


def test_paper_design_walks_counted(fp):
    """Walks of the paper's design (alias picks, one exact big move at each
    small node) through counting and top-k (fppr_aggregate): the top-k lists
    and digests of the oracle walker's endpoints."""
    import torch

    from test_gpu_alias import count_reference

    name, make, S, d, cap, alpha = CASES[0]
    g = make()
    say(f"case: big-move walks counted, {name}")
    G = fp.Graph(g, layout=fp.FPPR_LAYOUT_NARROW)
    P, al = G.alias_tables()
    sl = G.alias_slots(P, al)
    bm = G.big_moves(S, d, cap, alpha)
    src = np.arange(0, g.n, 7, dtype=np.uint32)
    ep, _ = fp.run_big_moves(G, sl, bm, S, alpha, 48, 31, sources=src, steps=False)
    o = fp.count(ep, 48, 12, sources=src, counts=False)
    torch.cuda.synchronize()
    ref_ep, _ = BM.run_with_alias(g.row_offsets, g.col, g.w, S, d, cap, fp.fppr_alpha_threshold(alpha), 31, 48, src)
    tk, dg = count_reference(ref_ep, src, 12)
    assert np.array_equal(o.topk.cpu().numpy().view(np.uint32), tk)
    assert np.array_equal(o.digest.cpu().numpy().view(np.uint64), dg)
