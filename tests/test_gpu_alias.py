"""Alias tables built on the GPU (Sec. 2.2, Algorithm 1) are bit-identical,
row by row, to the oracle's integer alias tables: every row of graphs with
hub rows of thousands of edges, weights up to 2^31 and unit weights, both
layouts; on the R-MAT scale-20 graph, the largest rows and a sample of the
rest. Walks that pick with the tables give the oracle's endpoints and steps
bit for bit. Build and walk times are printed."""
import sys

import numpy as np
import pytest

import counting_ref
import synth
from oracle import alias as A

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


def fetch(fp, G):
    import torch

    P, al = G.alias_tables()
    torch.cuda.synchronize()
    return P.cpu().numpy().view(np.uint64), al.cpu().numpy().view(np.uint32)


def rows_equal(g, P, al, rows):
    bad = []
    for v in rows:
        a, b = int(g.row_offsets[v]), int(g.row_offsets[v + 1])
        if a == b:
            continue
        Po, alo, _ = A.alias_table(g.w[a:b])
        if P[a:b].tolist() != Po or al[a:b].tolist() != alo:
            bad.append(int(v))
    return bad


CASES = {
    "chung-lu hubs": lambda: synth.chung_lu(3000, 60000, 2.05, 200, seed=5),
    "weights to 2^31": lambda: synth.chung_lu(2000, 30000, 2.2, 2_000_000_000, seed=6),
    "r-mat scale 12": lambda: synth.rmat(12, 16, .57, .19, .19, 10000, seed=7, zipf_s=1.2),
    "unit weights": lambda: synth.chung_lu(500, 4000, 2.1, 1, seed=8),
}


@pytest.mark.parametrize("name", list(CASES))
def test_alias_tables_equal_oracle(fp, name):
    g = CASES[name]()
    say(f"case: alias tables, {name}, n={g.n}, m={g.m}, max out-degree {g.degrees().max()}")
    layouts = [fp.FPPR_LAYOUT_WIDE]
    if int(g.w.max()) * int(g.degrees().max()) < 2**32:
        layouts.append(fp.FPPR_LAYOUT_NARROW)
    for lay in layouts:
        G = fp.Graph(g, layout=lay)
        P, al = fetch(fp, G)
        assert rows_equal(g, P, al, range(g.n)) == []
        # packed slots: threshold, own destination, the alias's destination
        import torch

        Pt, alt = G.alias_tables()
        sl = G.alias_slots(Pt, alt)
        torch.cuda.synchronize()
        sl = sl.cpu().numpy().view(np.uint64)
        rows = np.repeat(np.arange(g.n), g.degrees())
        first = g.row_offsets[:-1].astype(np.int64)[rows]
        assert np.array_equal(sl[:, 0], P)
        want = g.col.astype(np.uint64) | (g.col[first + al.astype(np.int64)].astype(np.uint64) << np.uint64(32))
        assert np.array_equal(sl[:, 1], want)
        if lay == fp.FPPR_LAYOUT_NARROW:
            # node records: row start, total | degree << 32
            ndr = G.alias_nodes()
            torch.cuda.synchronize()
            ndr = ndr.cpu().numpy().view(np.uint64)
            W = np.zeros(g.n, dtype=np.uint64)
            np.add.at(W, rows, g.w.astype(np.uint64))
            assert np.array_equal(ndr[:, 0], g.row_offsets[:-1].astype(np.uint64))
            assert np.array_equal(ndr[:, 1], W | (g.degrees().astype(np.uint64) << np.uint64(32)))
        # a second call on the same graph gives the same tables
        P2, al2 = fetch(fp, G)
        assert np.array_equal(P, P2) and np.array_equal(al, al2)


def test_alias_tables_scale20_sampled(fp):
    import torch

    g = synth.medium_graph()
    deg = g.degrees()
    say(f"case: alias tables, R-MAT scale 20, m={g.m}, max out-degree {deg.max()}")
    G = fp.Graph(g)
    G.alias_tables()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    P, al = G.alias_tables()
    t1.record()
    torch.cuda.synchronize()
    say(f"  alias tables of every row: {t0.elapsed_time(t1):.2f} ms")
    P = P.cpu().numpy().view(np.uint64)
    al = al.cpu().numpy().view(np.uint32)
    top = np.argsort(deg)[-64:]
    rng = np.random.default_rng(9)
    sample = rng.choice(np.flatnonzero(deg > 0), 4000, replace=False)
    assert rows_equal(g, P, al, np.concatenate([top, sample])) == []


@pytest.mark.parametrize("name", ["chung-lu hubs", "r-mat scale 12", "unit weights"])
def test_alias_walks_equal_oracle(fp, name):
    import torch

    g = CASES[name]()
    say(f"case: alias walks, {name}")
    G = fp.Graph(g, layout=fp.FPPR_LAYOUT_NARROW)
    P, al = G.alias_tables()
    sl = G.alias_slots(P, al)
    nd = G.alias_nodes()
    src = np.concatenate([np.arange(0, g.n, 37), [g.n - 1, 0, 0]]).astype(np.uint32)
    T = fp.fppr_alpha_threshold(0.15)
    ep, st = fp.run_alias(G, nd, sl, 0.15, 24, 123456789012, sources=src)
    torch.cuda.synchronize()
    ref_ep, ref_st = A.run(g.row_offsets, g.col, g.w, T, 123456789012, 24, src)
    assert np.array_equal(ep.cpu().numpy().view(np.uint32).reshape(len(src), 24), ref_ep)
    assert np.array_equal(st.cpu().numpy().view(np.uint32).reshape(len(src), 24), ref_st)


def test_alias_walks_edges(fp):
    import torch

    g = CASES["unit weights"]()
    say("case: alias walks, invalid source, all nodes, wide graph refused")
    G = fp.Graph(g, layout=fp.FPPR_LAYOUT_NARROW)
    P, al = G.alias_tables()
    sl = G.alias_slots(P, al)
    nd = G.alias_nodes()
    src = np.array([3, g.n, 7], dtype=np.uint32)
    ep, st = fp.run_alias(G, nd, sl, 0.3, 5, 1, sources=src)
    torch.cuda.synchronize()
    e = ep.cpu().numpy().view(np.uint32).reshape(3, 5)
    assert np.all(e[1] == 0xFFFFFFFF) and np.all(st.cpu().numpy().reshape(3, 5)[1] == 0)
    ref_ep, _ = A.run(g.row_offsets, g.col, g.w, fp.fppr_alpha_threshold(0.3), 1, 5, [3, 7])
    assert np.array_equal(e[[0, 2]], ref_ep)
    ep_all, _ = fp.run_alias(G, nd, sl, 0.3, 2, 1, steps=False)
    torch.cuda.synchronize()
    ref_all, _ = A.run(g.row_offsets, g.col, g.w, fp.fppr_alpha_threshold(0.3), 1, 2, range(g.n))
    assert np.array_equal(ep_all.cpu().numpy().view(np.uint32).reshape(g.n, 2), ref_all)
    Gw = fp.Graph(g, layout=fp.FPPR_LAYOUT_WIDE)
    Pw, alw = Gw.alias_tables()
    with pytest.raises(fp.FpprError):
        fp.run_alias(Gw, nd, Gw.alias_slots(Pw, alw), 0.3, 5, 1, sources=src)
    with pytest.raises(fp.FpprError):
        fp.run_alias(G, nd, sl, 1.5, 5, 1, sources=src)


def test_alias_walks_scale20(fp):
    """R-MAT scale 20, R = 16 walks from every node: timed, and 512 sampled
    sources recomputed by the oracle."""
    import torch

    g = synth.medium_graph()
    say("case: alias walks, R-MAT scale 20, R = 16 from every node")
    G = fp.Graph(g)
    assert G.layout() == fp.FPPR_LAYOUT_NARROW
    P, al = G.alias_tables()
    sl = G.alias_slots(P, al)
    nd = G.alias_nodes()
    fp.run_alias(G, nd, sl, 0.15, 16, 3)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    ep, st = fp.run_alias(G, nd, sl, 0.15, 16, 3)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    steps = int(st.to(torch.int64).sum().item())
    say(f"  {g.n * 16} walks, {steps} steps in {ms:.2f} ms: {steps / ms * 1e3:.3e} walk-steps/s")
    # the same walks on the library's prefix-sum path (no stitching), for
    # comparison: walk time from the stage timer, steps from its statistics
    prm = fp.make_params(0.15, 16, 3, 1, False, False, True, True)
    ws = torch.empty((fp.fppr_plan(G, prm, g.n) + 7) // 8, dtype=torch.int64, device="cuda")
    for _ in range(2):
        out = fp.alloc_outputs(g.n, 16, 1, counts=False, digests=True, stats=True)
        prof = fp.Profile()
        out.profile = prof
        fp.fppr_run(G, prm, None, g.n, ws, out, None)
        torch.cuda.synchronize()
    walk_ms, _ = prof.read()
    cdf_steps = out.stats_dict()["steps"]
    say(f"  prefix-sum path: {cdf_steps} steps, walk phase {walk_ms:.2f} ms: "
        f"{cdf_steps / walk_ms * 1e3:.3e} walk-steps/s")
    # coins depend on (walk, move, source) only, so every walk has the same
    # number of moves, and here of steps, whichever edges it picks
    assert cdf_steps == steps
    rng = np.random.default_rng(4)
    sample = np.sort(rng.choice(g.n, 512, replace=False))
    e = ep.cpu().numpy().view(np.uint32).reshape(g.n, 16)[sample]
    s_ = st.cpu().numpy().view(np.uint32).reshape(g.n, 16)[sample]
    ref_ep, ref_st = A.run(g.row_offsets, g.col, g.w, fp.fppr_alpha_threshold(0.15), 3, 16, sample)
    assert np.array_equal(e, ref_ep) and np.array_equal(s_, ref_st)


def test_alias_walks_scale24_ab(fp):
    """R-MAT scale 24 (the benchmark graph), R = 16 from every node, no
    stitching: alias walks against the prefix-tree path on the same walks
    (equal step counts, since coins do not depend on the picks), both timed;
    288 sampled walks (hub sources included) recomputed by the oracle."""
    import torch

    g = synth.scale24_graph()
    say(f"case: alias walks, R-MAT scale 24 (n={g.n}, m={g.m}), R = 16 from every node")
    G = fp.Graph(g)
    assert G.layout() == fp.FPPR_LAYOUT_NARROW
    P, al = G.alias_tables()
    sl = G.alias_slots(P, al)
    nd = G.alias_nodes()
    del P, al
    fp.run_alias(G, nd, sl, 0.15, 16, 3, steps=False)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    ep, st = fp.run_alias(G, nd, sl, 0.15, 16, 3)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    steps = int(st.to(torch.int64).sum().item())
    say(f"  alias walks: {steps} steps in {ms:.2f} ms: {steps / ms * 1e3:.3e} walk-steps/s")
    prm = fp.make_params(0.15, 16, 3, 1, False, False, True, True)
    ws = torch.empty((fp.fppr_plan(G, prm, g.n) + 7) // 8, dtype=torch.int64, device="cuda")
    for _ in range(2):
        out = fp.alloc_outputs(g.n, 16, 1, counts=False, digests=True, stats=True)
        prof = fp.Profile()
        out.profile = prof
        fp.fppr_run(G, prm, None, g.n, ws, out, None)
        torch.cuda.synchronize()
    walk_ms, _ = prof.read()
    kern_ms, _ = prof.read_walk()
    cdf_steps = out.stats_dict()["steps"]
    say(f"  prefix-tree path: {cdf_steps} steps, walk phase {walk_ms:.2f} ms (walk kernel {kern_ms:.2f} ms): "
        f"{cdf_steps / walk_ms * 1e3:.3e} walk-steps/s")
    assert cdf_steps == steps
    # 288 walks recomputed by the oracle: 6 walks from each of the 8 largest
    # rows (hubs of up to 370,930 edges) and of 40 random nodes with out-edges
    deg = g.degrees()
    rng = np.random.default_rng(24)
    src = np.unique(np.concatenate([np.argsort(deg)[-8:],
                                    rng.choice(np.flatnonzero(deg > 0), 40, replace=False)])).astype(np.uint32)
    e = ep.cpu().numpy().view(np.uint32).reshape(g.n, 16)[src, :6]
    s_ = st.cpu().numpy().view(np.uint32).reshape(g.n, 16)[src, :6]
    ref_ep, ref_st = A.run(g.row_offsets, g.col, g.w, fp.fppr_alpha_threshold(0.15), 3, 6, src)
    assert np.array_equal(e, ref_ep) and np.array_equal(s_, ref_st)


def count_reference(ep, sources, k):
    topk, digest, _, _ = counting_ref.count_reference(ep, sources, k)
    return topk, digest


def test_aggregate_equals_run_counting(fp):
    """fppr_aggregate over fppr_run's own endpoints gives fppr_run's counts,
    top-k and digests (sort path with counts, and the hash path of R > 256)."""
    import torch

    g = CASES["chung-lu hubs"]()
    say("case: fppr_aggregate over fppr_run's endpoints")
    G = fp.Graph(g)
    src = np.arange(0, g.n, 11, dtype=np.uint32)
    for R, k, counts in ((100, 16, True), (5000, 32, False)):
        o = fp.run(G, 0.15, R, 77, sources=src, topk=k, counts=counts, endpoints=True)
        a = fp.count(o.endpoints.reshape(-1), R, k, sources=src, counts=counts)
        torch.cuda.synchronize()
        assert torch.equal(a.topk, o.topk) and torch.equal(a.digest, o.digest)
        if counts:
            assert torch.equal(a.counts, o.counts) and torch.equal(a.n_distinct, o.n_distinct)


def test_alias_walks_counted(fp):
    """Alias walks (the paper's picks) through counting and top-k: the top-k
    lists and digests of the oracle walker's endpoints."""
    import torch

    g = CASES["r-mat scale 12"]()
    say("case: alias walks counted")
    G = fp.Graph(g, layout=fp.FPPR_LAYOUT_NARROW)
    P, al = G.alias_tables()
    sl = G.alias_slots(P, al)
    nd = G.alias_nodes()
    src = np.arange(0, g.n, 29, dtype=np.uint32)
    ep, _ = fp.run_alias(G, nd, sl, 0.15, 64, 5, sources=src, steps=False)
    o = fp.count(ep, 64, 16, sources=src, counts=False)
    torch.cuda.synchronize()
    ref_ep, _ = A.run(g.row_offsets, g.col, g.w, fp.fppr_alpha_threshold(0.15), 5, 64, src)
    tk, dg = count_reference(ref_ep, src, 16)
    assert np.array_equal(o.topk.cpu().numpy().view(np.uint32), tk)
    assert np.array_equal(o.digest.cpu().numpy().view(np.uint64), dg)


def test_alias_slots_of_long_rows_scale20(fp):
    """Packed slots (threshold, own destination, alias's destination) of the
    64 largest rows of R-MAT scale 20 (up to 69,306 edges: lanes loop over
    the row) and 4,000 sampled rows, against the oracle's tables."""
    import torch

    g = synth.medium_graph()
    deg = g.degrees()
    say("case: alias slots of long rows, R-MAT scale 20")
    G = fp.Graph(g)
    Pt, alt = G.alias_tables()
    sl = G.alias_slots(Pt, alt)
    torch.cuda.synchronize()
    sl = sl.cpu().numpy().view(np.uint64)
    rng = np.random.default_rng(19)
    rows = np.concatenate([np.argsort(deg)[-64:], rng.choice(np.flatnonzero(deg > 0), 4000, replace=False)])
    for v in rows:
        a, b = int(g.row_offsets[v]), int(g.row_offsets[v + 1])
        Po, alo, _ = A.alias_table(g.w[a:b])
        want = g.col[a:b].astype(np.uint64) | (g.col[a + np.asarray(alo, dtype=np.int64)].astype(np.uint64)
                                                << np.uint64(32))
        assert np.array_equal(sl[a:b, 0], np.asarray(Po, dtype=np.uint64)), v
        assert np.array_equal(sl[a:b, 1], want), v
