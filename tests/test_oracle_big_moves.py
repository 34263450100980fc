"""Pins of the exact big-move oracle (Sec. 4.2, Algorithm 4, Example 5,
Lemma 2) against what the paper and the mathematics fix.

A plausible mistake in it fails one of these: a dropped (1 - alpha) factor or
a coin on the wrong side of a step (Example 5's printed values, Lemma 2's
masses, brute-force path enumeration), lost mass at nodes without
out-neighbours (brute force, unit mass, the chain test), a wrong stop rule
(hand-worked stop cases), a wrong expansion or aggregation index (brute
force, the chain test against plain PPR), a fixed-point product in the wrong
order or rounded the wrong way (the dyadic case must be exact, error bound,
edge-order invariance), and a distribution that is not the one the sampled
short walks follow (chi-square against the C oracle's pool at a fixed
length)."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from exact_ppr import _series, ppr_exact, transition
from oracle import big_moves as BM
from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def csr(n, edges, weights=None):
    """Plain CSR in the given edge order (rows by source, order kept)."""
    w = [1] * len(edges) if weights is None else list(weights)
    order = sorted(range(len(edges)), key=lambda i: edges[i][0])
    off = np.zeros(n + 1, dtype=np.uint64)
    for u, _ in edges:
        off[u + 1] += 1
    off = np.cumsum(off).astype(np.uint64)
    col = np.array([edges[i][1] for i in order], dtype=np.uint32)
    wt = np.array([w[i] for i in order], dtype=np.uint32)
    return off, col, wt


def random_graph(n, m, seed, dangling=0.0, wmax=9):
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m)
    keep = rng.random(n) >= dangling
    src = src[keep[src]]
    dst = rng.integers(0, n, src.size)
    edges = list(zip(src.tolist(), dst.tolist()))
    return csr(n, edges, rng.integers(1, wmax + 1, len(edges)).tolist())


def brute(off, col, w, v, alpha, k):
    """Every walk from v of at most k steps, one path at a time (each edge a
    separate branch), with its probability; a walk arriving at t after j
    steps stops there with alpha (terminated outcome) and otherwise is an
    active outcome if j = k or t has no out-neighbours."""
    al = Fraction(alpha)
    out = {}

    def add(key, p):
        out[key] = out.get(key, 0) + p

    def rec(u, j, p):
        add((u, j, 1), al * p)
        cont = (1 - al) * p
        a, b = int(off[u]), int(off[u + 1])
        if j == k or a == b:
            add((u, j, 0), cont)
            return
        Wu = sum(int(x) for x in w[a:b])
        for e in range(a, b):
            rec(int(col[e]), j + 1, cont * Fraction(int(w[e]), Wu))

    a, b = int(off[v]), int(off[v + 1])
    Wv = sum(int(x) for x in w[a:b])
    for e in range(a, b):
        rec(int(col[e]), 1, Fraction(int(w[e]), Wv))
    return {key: p for key, p in out.items() if p != 0}


def longest(bm):
    return max(j for _, j, _ in bm)


# --------------------------------------------------------------------------
# Example 5 and Lemma 2
# --------------------------------------------------------------------------
def test_example5_exact_values():
    fx = json.load(open(os.path.join(GOLDEN, "example5_big_moves.json")))
    off, col, w = csr(5, [tuple(e) for e in fx["edges"]] + [(0, 1), (1, 0)])
    bm = BM.big_moves_exact(off, col, w, fx["source"], Fraction(fx["alpha"]), d=4)
    assert longest(bm) == fx["steps"]
    by_mark = {}
    for (t, _, mark), p in bm.items():
        by_mark[(t, mark)] = by_mark.get((t, mark), 0) + p
    want = {(b["end"], 1 if b["terminated"] else 0): Fraction(b["p"]) for b in fx["big_moves"]}
    assert by_mark == want
    want_len = {(t, L, 1 if term else 0): Fraction(p) for t, L, term, p in fx["derived_by_length"]["entries"]}
    assert bm == want_len
    # every probability in the example is dyadic, so the 62-bit form is exact
    fixed = BM.big_moves_fixed(off, col, w, fx["source"], 1 << 31, d=4)
    assert fixed == {key: int(p * BM.ONE) for key, p in bm.items()}


@pytest.mark.parametrize("alpha,d,seed", [(Fraction(1, 5), 8, 1), (Fraction(1, 2), 16, 2),
                                          (Fraction(3, 20), 32, 3), (Fraction(9, 10), 6, 4)])
def test_lemma2_unit_mass(alpha, d, seed):
    """Graphs where every node has out-neighbours: the big moves of every node
    sum to exactly 1, the terminated part is 1 - (1 - alpha)^k, the active part
    (1 - alpha)^k, and every active outcome has length k."""
    n = 40
    rng = np.random.default_rng(seed)
    edges = [(u, int(t)) for u in range(n) for t in rng.integers(0, n, rng.integers(1, 4))]
    off, col, w = csr(n, edges, rng.integers(1, 7, len(edges)).tolist())
    ks = set()
    for v in range(n):
        bm = BM.big_moves_exact(off, col, w, v, alpha, d)
        k = longest(bm)
        ks.add(k)
        assert sum(bm.values()) == 1
        term = sum(p for (_, _, m), p in bm.items() if m == 1)
        assert term == 1 - (1 - alpha) ** k
        assert all(j == k for (_, j, m) in bm if m == 0)
    assert len(ks) > 1  # the stop rule gives different depths


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_paths(seed):
    """Random tiny graphs with parallel edges, self loops and nodes without
    out-neighbours: the frontier expansion equals the enumeration of every
    path, at the depth the stop rule chose and at fixed depths."""
    off, col, w = random_graph(9, 22, seed, dangling=0.25)
    alpha = Fraction(1, 3 + seed)
    for v in range(9):
        if off[v] == off[v + 1]:
            continue
        for d in (3, 5, 9, 40):
            bm = BM.big_moves_exact(off, col, w, v, alpha, d)
            assert bm == brute(off, col, w, v, alpha, longest(bm))
            assert sum(bm.values()) == 1
        for L in (1, 2, 4):
            assert BM.big_moves_exact(off, col, w, v, alpha, 0, fixed_k=L) == brute(off, col, w, v, alpha, L)


def test_stop_rule_cases():
    a = Fraction(1, 4)
    # |B| + |F| = 2 deg >= d at once: one plain step, no expansion
    off, col, w = csr(3, [(0, 1), (0, 2), (1, 0), (2, 0)])
    bm = BM.big_moves_exact(off, col, w, 0, a, d=4)
    assert bm == {(1, 1, 1): a / 2, (2, 1, 1): a / 2, (1, 1, 0): (1 - a) / 2, (2, 1, 0): (1 - a) / 2}
    # a 10-cycle: B gains one node per level, so the size bound stops it at
    # |B| + |F| = k + 1 >= d, and with a large d it stops one level after B
    # has every node (the level that reached no new node)
    off, col, w = csr(10, [(i, (i + 1) % 10) for i in range(10)])
    assert longest(BM.big_moves_exact(off, col, w, 0, a, d=6)) == 5
    assert longest(BM.big_moves_exact(off, col, w, 0, a, d=100)) == 11
    # an out-neighbour without out-neighbours: its continuing mass is an
    # active outcome of length 1, and nothing new is reached, so it stops
    off, col, w = csr(2, [(0, 1)])
    assert BM.big_moves_exact(off, col, w, 0, a, d=8) == {(1, 1, 1): a, (1, 1, 0): 1 - a}
    # frozen entries count towards the size bound: 0 -> {1, 2}, 1 without
    # out-neighbours, 2 -> 3 -> 0. After one expansion B = {1, 2, 3}, F = {3}
    # and the frozen entry at 1 make 5 >= d = 5 (without the frozen entry
    # it would be 4 < 5 and a third level would follow)
    off, col, w = csr(4, [(0, 1), (0, 2), (2, 3), (3, 0)])
    bm = BM.big_moves_exact(off, col, w, 0, a, d=5)
    assert longest(bm) == 2 and (1, 1, 0) in bm and (3, 2, 0) in bm
    # a node without out-neighbours has no big moves
    with pytest.raises(ValueError):
        BM.big_moves_exact(off, col, w, 1, a, d=8)


# --------------------------------------------------------------------------
# fixed point
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(4))
def test_fixed_point_close_to_exact_and_order_free(seed):
    off, col, w = random_graph(30, 90, 10 + seed, dangling=0.2, wmax=10000)
    T = O.alpha_threshold(0.15)
    alpha = Fraction(T, 1 << 32)
    rng = np.random.default_rng(seed)
    # the same rows with their edges in another order
    col2, w2 = col.copy(), w.copy()
    for u in range(30):
        a, b = int(off[u]), int(off[u + 1])
        p = rng.permutation(b - a) + a
        col2[a:b], w2[a:b] = col[p], w[p]
    for v in range(30):
        if off[v] == off[v + 1]:
            continue
        ex = BM.big_moves_exact(off, col, w, v, alpha, 24)
        fx = BM.big_moves_fixed(off, col, w, v, T, 24)
        assert set(fx) <= set(ex)
        # each floor loses under one unit; an outcome gathers at most a few
        # thousand floors on graphs this size
        for key, p in ex.items():
            assert abs(Fraction(fx.get(key, 0), BM.ONE) - p) < Fraction(1, 1 << 48)
        tot = sum(fx.values())
        assert BM.ONE - (1 << 20) < tot <= BM.ONE
        assert BM.big_moves_fixed(off, col2, w2, v, T, 24) == fx


def test_table_and_pick():
    off, col, w = csr(5, [(0, 1), (0, 2), (0, 2), (1, 3), (2, 4), (3, 0), (4, 0)], [1, 2, 3, 1, 1, 1, 1])
    T = 1 << 30
    offs, ent, wts = BM.table(off, col, w, [0, 1, 3], T, d=6)
    assert offs[0] == 0 and offs[-1] == ent.size == wts.size
    for r, v in enumerate((0, 1, 3)):
        e = ent[offs[r]:offs[r + 1]]
        q = wts[offs[r]:offs[r + 1]]
        assert np.all(np.diff(e.astype(object)) > 0)
        bm = BM.big_moves_fixed(off, col, w, v, T, d=6)
        assert {BM.encode(*k): x for k, x in bm.items()} == dict(zip(e.tolist(), q.tolist()))
        # pick: D = 0 takes the first entry, D = 2^64 - 1 the last; a draw
        # just at an entry's prefix boundary takes the next entry
        assert BM.pick(e, q, 0) == int(e[0])
        assert BM.pick(e, q, (1 << 64) - 1) == int(e[-1])
        tot = int(q.astype(object).sum())
        acc = 0
        for i in range(len(e) - 1):
            acc += int(q[i])
            D = -((-acc << 64) // tot)  # smallest D with floor(D * tot / 2^64) = acc
            assert BM.pick(e, q, D) == int(e[i + 1])
            assert BM.pick(e, q, D - 1) == int(e[i])


# --------------------------------------------------------------------------
# the two things exact big moves are for
# --------------------------------------------------------------------------
def chain_with_big_moves(n, off, col, w, alpha, sources, small, d, cap=None):
    P, dang = transition(n, off, col, w)
    Q = ((1.0 - float(alpha)) * P).tolil()
    A = (float(alpha) * P).tolil()
    for v in small:
        Q.rows[v], Q.data[v], A.rows[v], A.data[v] = [], [], [], []
        for (t, _, mark), p in BM.big_moves_exact(off, col, w, int(v), alpha, d, max_entries=cap).items():
            M = A if mark == 1 else Q
            M[v, t] = M[v, t] + float(p)
    return _series(n, sources, Q.tocsr(), A.tocsr(), dang, float(alpha))


@pytest.mark.parametrize("seed", range(4))
def test_size_look_ahead(seed):
    """With the size look-ahead every table holds at most max(cap, 2 deg(v))
    entries, is still the exact distribution of every walk of its depth
    (brute force), and never goes deeper than without the cap."""
    off, col, w = random_graph(12, 40, 20 + seed, dangling=0.15)
    alpha = Fraction(1, 4)
    for v in range(12):
        deg = int(off[v + 1]) - int(off[v])
        if deg == 0:
            continue
        free = BM.big_moves_exact(off, col, w, v, alpha, 64)
        for cap in (2, 6, 12, 30):
            bm = BM.big_moves_exact(off, col, w, v, alpha, 64, max_entries=cap)
            assert len(bm) <= max(cap, 2 * deg)
            assert longest(bm) <= longest(free)
            assert bm == brute(off, col, w, v, alpha, longest(bm))
            fx = BM.big_moves_fixed(off, col, w, v, 1 << 30, 64, max_entries=cap)
            assert set(fx) <= set(BM.big_moves_exact(off, col, w, v, Fraction(1, 4), 64, max_entries=cap))
    # a node in front of a 10-edge row: a cap of 8 keeps it at one step
    off, col, w = csr(12, [(0, 1)] + [(1, t) for t in range(2, 12)])
    assert longest(BM.big_moves_exact(off, col, w, 0, alpha, 64, max_entries=8)) == 1
    assert longest(BM.big_moves_exact(off, col, w, 0, alpha, 64, max_entries=22)) == 2


@pytest.mark.parametrize("d,cap", [(4, None), (16, None), (64, None), (64, 24)])
def test_walks_on_big_moves_give_plain_ppr(d, cap):
    """A walk that takes one big move at every small node and plain steps
    elsewhere ends with exactly the PPR distribution of plain walks
    (Lemma 2: a big move is the exact distribution of the walk's next k
    steps), on a graph with nodes without out-neighbours."""
    g = synth.chung_lu(300, 1500, 2.3, 50, seed=77)
    off, col, w = g.row_offsets, g.col, g.w
    deg = g.degrees()
    assert (deg == 0).any()
    small = np.flatnonzero((deg >= 1) & (deg <= 8))
    alpha = Fraction(3, 20)
    src = np.arange(0, 300, 7)
    pi = ppr_exact(g.n, off, col, w, 0.15, src)
    chain = chain_with_big_moves(g.n, off, col, w, alpha, src, small, d, cap)
    assert np.max(np.abs(chain - pi)) < 1e-12
    assert np.allclose(chain.sum(axis=1), 1.0, atol=1e-12)


def test_matches_sampled_pool_at_fixed_length():
    """At the pool's fixed length L the exact outcome distribution is the one
    the C oracle's sampled short walks follow (chi-square over K = 2^16 slots
    per node; rare outcomes merged)."""
    from scipy.stats import chisquare

    g = synth.chung_lu(400, 1600, 2.3, 20, seed=78)
    deg = g.degrees()
    small = np.flatnonzero((deg >= 1) & (deg <= 4))
    K, L = 1 << 16, 3
    T = O.alpha_threshold(0.3)
    pool = O.Pool(O.Graph(g.n, g.row_offsets, g.col, g.w), S=4, L=L, K=K, alpha=0.3, seed=11)
    ent = pool.entries().reshape(small.size, K)
    alpha = Fraction(T, 1 << 32)
    pvals = []
    for r in range(0, small.size, max(1, small.size // 12)):
        v = int(small[r])
        ex = BM.big_moves_exact(g.row_offsets, g.col, g.w, v, alpha, 0, fixed_k=L)
        keys = sorted(ex, key=lambda k: BM.encode(*k))
        enc = [BM.encode(*k) for k in keys]
        obs = {e: 0 for e in enc}
        for e in ent[r].tolist():
            assert e in obs, (v, e)
            obs[e] += 1
        exp = np.array([float(ex[k]) * K for k in keys])
        o = np.array([obs[e] for e in enc], dtype=float)
        big = exp >= 5
        o2 = np.append(o[big], o[~big].sum())
        e2 = np.append(exp[big], exp[~big].sum())
        if e2[-1] == 0:
            o2, e2 = o2[:-1], e2[:-1]
        if o2.size > 1:
            pvals.append(chisquare(o2, e2).pvalue)
    assert len(pvals) >= 8
    assert min(pvals) > 1e-5


# --------------------------------------------------------------------------
# walks that take big moves
# --------------------------------------------------------------------------
def test_walk_without_small_nodes_is_the_plain_walk():
    """With no big-move tables the Python walk is the C oracle's plain walk,
    endpoint for endpoint and step for step."""
    g = synth.chung_lu(200, 900, 2.3, 30, seed=79)
    G = O.Graph(g.n, g.row_offsets, g.col, g.w)
    src = np.arange(0, 200, 9, dtype=np.uint32)
    ref = O.run(G, 0.2, 40, 17, sources=src, want_endpoints=True, want_lengths=True, want_counts=False)
    ep, ln = BM.run(G, {}, O.alpha_threshold(0.2), 17, 40, src)
    assert np.array_equal(ep, ref.endpoints) and np.array_equal(ln, ref.lengths)


def test_walks_with_big_moves_estimate_plain_ppr():
    """Walks that take big moves at small nodes (out-degree <= 6) estimate
    the plain PPR without bias (binomial z-check of every (source, node)
    pair with enough expected walks), and their lengths follow the plain
    walk's law P(len = l) = alpha (1 - alpha)^(l - 1)."""
    from scipy.stats import chisquare

    g = synth.chung_lu(120, 500, 2.3, 20, seed=80)
    G = O.Graph(g.n, g.row_offsets, g.col, g.w)
    T = O.alpha_threshold(0.25)
    a = T / 2.0**32
    tables = BM.tables_by_node(g.row_offsets, g.col, g.w, 6, T, 24)
    assert len(tables) > 40
    src = np.array([0, 3, 11, 40, 77], dtype=np.uint32)
    R = 3000
    ep, ln = BM.run(G, tables, T, 5, R, src)
    pi = ppr_exact(g.n, g.row_offsets, g.col, g.w, a, src)
    from exact_ppr import mc_z_check

    dense = np.zeros((len(src), g.n), dtype=np.int64)
    for r in range(len(src)):
        np.add.at(dense[r], ep[r].astype(np.int64), 1)
    ok, info = mc_z_check(dense, pi, R)
    assert ok, info
    L = ln.ravel().astype(np.int64)
    top = 12
    obs = np.array([np.count_nonzero(L == l) for l in range(1, top)] + [np.count_nonzero(L >= top)])
    p = np.array([a * (1 - a) ** (l - 1) for l in range(1, top)] + [(1 - a) ** (top - 1)])
    assert chisquare(obs, p * L.size).pvalue > 1e-4


def test_paper_design_walk_estimates_plain_ppr():
    """Walks of the paper's design (alias picks, one exact big move at each
    small node) estimate the plain PPR without bias and keep the geometric
    length law; with S = 0 (no small nodes) they are the alias walks."""
    from scipy.stats import chisquare

    from exact_ppr import mc_z_check
    from oracle import alias as A

    g = synth.chung_lu(120, 500, 2.3, 20, seed=82)
    T = O.alpha_threshold(0.25)
    a = T / 2.0**32
    src = np.array([0, 3, 11, 40, 77], dtype=np.uint32)
    R = 3000
    ep, ln = BM.run_with_alias(g.row_offsets, g.col, g.w, 6, 24, 64, T, 5, R, src)
    pi = ppr_exact(g.n, g.row_offsets, g.col, g.w, a, src)
    dense = np.zeros((len(src), g.n), dtype=np.int64)
    for r in range(len(src)):
        np.add.at(dense[r], ep[r].astype(np.int64), 1)
    ok, info = mc_z_check(dense, pi, R)
    assert ok, info
    L = ln.ravel().astype(np.int64)
    top = 12
    obs = np.array([np.count_nonzero(L == l) for l in range(1, top)] + [np.count_nonzero(L >= top)])
    p = np.array([a * (1 - a) ** (l - 1) for l in range(1, top)] + [(1 - a) ** (top - 1)])
    assert chisquare(obs, p * L.size).pvalue > 1e-4
    e0, l0 = BM.run_with_alias(g.row_offsets, g.col, g.w, 0, 24, 64, T, 5, 40, src)
    e1, l1 = A.run(g.row_offsets, g.col, g.w, T, 5, 40, src)
    assert np.array_equal(e0, e1) and np.array_equal(l0, l1)
