"""Pins of the alias-table and alias-tree oracle (Sec. 2.2, Algorithm 1,
Example 2; Sec. 4.1, Algorithm 3, Examples 3-4, Lemma 1).

A plausible mistake fails one of these: a wrong update of the large item or
a swapped x / y (Example 2's printed p and a, the exact selection formula),
items stranded in S^l (range invariant and the exact selection formula), a slot / threshold split
of the draw that is not uniform (enumeration of every draw value), a subset
weight or a level wired to the wrong group (Examples 3-4, Lemma 1 by exact
enumeration through the tree, for contiguous and random partitions), a tree
deeper than ceil(log_d n)."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import alias as A

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dec(x):
    """A printed decimal as an exact fraction."""
    return Fraction(str(x))


def fixture():
    return json.load(open(os.path.join(GOLDEN, "examples_2_3_4_alias.json")))


def table_probs(P, al, W):
    """Selection probability of every item from a table (the formula below
    Algorithm 1: own slot with p, every slot aliased to it with 1 - p)."""
    n = len(P)
    pr = [Fraction(0)] * n
    for i in range(n):
        pr[i] += Fraction(P[i], n * W)
        pr[al[i]] += Fraction(W - P[i], n * W)
    return pr


def D_for(X, N):
    """Smallest 64-bit D with floor(D N / 2^64) = X."""
    return -((-X << 64) // N)


def test_example2():
    fx = fixture()["example2"]
    P, al, W = A.alias_table(fx["weights"])
    n = len(fx["weights"])
    assert [Fraction(n * x, W) for x in fx["weights"]] == [dec(p) for p in fx["initial_p"]]
    assert [Fraction(p, W) for p in P] == [dec(p) for p in fx["p"]]
    assert al == fx["alias"]


def test_examples3_4():
    fx = fixture()["examples3_4"]
    levels = A.alias_tree(fx["weights"], fx["d"])
    assert len(levels) == 2
    leaves, root = levels
    W = sum(fx["weights"])
    assert [Fraction(g[3], W) for g in leaves] == [dec(x) for x in fx["subset_weight_fractions"]]
    members, P, al, Wr = root[0]
    assert Wr == W and members == [0, 1]
    assert [Fraction(p, Wr) for p in P] == [dec(p) for p in fx["root_p"]]
    assert al == fx["root_alias"]
    assert table_probs(P, al, Wr)[0] == dec(fx["prob_S1"])
    # the first leaf is Example 2's table
    ex2 = fixture()["example2"]
    assert leaves[0][2] == ex2["alias"]


@pytest.mark.parametrize("seed", range(8))
def test_alias_table_exact(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 60))
    w = rng.integers(1, [2, 10, 1000, 2**31][seed % 4], n).tolist()
    P, al, W = A.alias_table(w)
    assert W == sum(w)
    assert all(0 <= p <= W for p in P)
    assert all(al[i] == i for i in range(n) if P[i] == W)
    assert table_probs(P, al, W) == [Fraction(x, W) for x in w]


@pytest.mark.parametrize("w", [[1], [1, 1], [3, 1], [1, 2, 3, 4], [5, 1, 1, 1, 1, 1, 7], [2, 9, 4, 1, 1]])
def test_every_draw_value(w):
    """All n W values of X: each item is chosen for exactly n w(e) of them,
    and the 64-bit draw at each X's lower edge lands on that X."""
    P, al, W = A.alias_table(w)
    n = len(w)
    N = n * W
    cnt = [0] * n
    for X in range(N):
        i, U = divmod(X, W)
        e = i if U < P[i] else al[i]
        cnt[e] += 1
        D = D_for(X, N)
        assert A.alias_pick(P, al, W, D) == e
        if D > 0:
            assert (D - 1) * N >> 64 == X - 1
    assert cnt == [n * x for x in w]
    assert A.alias_pick(P, al, W, 2**64 - 1) == (n - 1 if P[n - 1] == W else al[n - 1])


def tree_probs(levels):
    """Exact probability of every original item through the tree: the
    product of the table probabilities along its root-to-leaf path."""
    out = {}

    def down(depth, g, p):
        level = levels[len(levels) - 1 - depth]
        members, P, al, W = level[g]
        for j, q in enumerate(table_probs(P, al, W)):
            if depth == len(levels) - 1:
                out[members[j]] = out.get(members[j], 0) + p * q
            else:
                down(depth + 1, members[j], p * q)

    down(0, 0, Fraction(1))
    return out


def random_split(seed):
    def split(n, d):
        perm = np.random.default_rng(seed + n).permutation(n).tolist()
        return [sorted(perm[a:a + d]) for a in range(0, n, d)]
    return split


@pytest.mark.parametrize("n,d", [(1, 2), (7, 2), (6, 3), (50, 3), (200, 8), (1000, 16), (33, 32)])
@pytest.mark.parametrize("how", ["contiguous", "random"])
def test_lemma1(n, d, how):
    """Lemma 1: through the tree an item is chosen with probability w / W,
    for any partition; the tree has ceil(log_d n) levels below the root
    (one level when n <= d)."""
    rng = np.random.default_rng(n * 31 + d)
    w = rng.integers(1, 1000, n).tolist()
    split = A.contiguous_split if how == "contiguous" else random_split(n + d)
    levels = A.alias_tree(w, d, split)
    W = sum(w)
    assert tree_probs(levels) == {e: Fraction(x, W) for e, x in enumerate(w)}
    h = 1
    while d ** h < n:
        h += 1
    assert len(levels) == h


def test_tree_pick_enumerated():
    """alias_tree_pick over every (root X, leaf X) pair of Examples 3-4's
    tree, weighted by each pair's probability, gives w / W exactly."""
    w = fixture()["examples3_4"]["weights"]
    levels = A.alias_tree(w, 3)
    leaves, root = levels
    _, Pr, alr, Wr = root[0]
    Nr = len(Pr) * Wr
    got = {}
    for Xr in range(Nr):
        g = root[0][0][A.alias_pick(Pr, alr, Wr, D_for(Xr, Nr))]
        members, P, al, W = leaves[g]
        N = len(P) * W
        for X in range(N):
            e = A.alias_tree_pick(levels, [D_for(Xr, Nr), D_for(X, N)])
            got[e] = got.get(e, 0) + Fraction(1, Nr * N)
    assert got == {e: Fraction(x, sum(w)) for e, x in enumerate(w)}


def test_rejects_bad_input():
    with pytest.raises(ValueError):
        A.alias_table([])
    with pytest.raises(ValueError):
        A.alias_table([1, 0, 2])
    with pytest.raises(ValueError):
        A.alias_tree([1, 2, 3], 1)


# --------------------------------------------------------------------------
# walks that pick with alias tables
# --------------------------------------------------------------------------
def test_alias_walk_is_the_plain_walk_on_single_edge_rows():
    """Where every row has one edge (or none) both picks are forced, so the
    alias walk is the C oracle's plain walk, endpoint for endpoint and step
    for step (same draws, coins, restarts)."""
    import synth
    from oracle import oracle as O

    rng = np.random.default_rng(12)
    n = 300
    src = np.flatnonzero(rng.random(n) < 0.85).astype(np.uint32)
    dst = rng.integers(0, n, src.size).astype(np.uint32)
    g = synth.csr_from_edges(n, src, dst, rng.integers(1, 50, src.size).astype(np.uint32))
    T = O.alpha_threshold(0.1)
    sources = np.arange(0, n, 7, dtype=np.uint32)
    ref = O.run(O.Graph(g.n, g.row_offsets, g.col, g.w), 0.1, 24, 31, sources=sources,
                want_endpoints=True, want_lengths=True, want_counts=False)
    ep, ln = A.run(g.row_offsets, g.col, g.w, T, 31, 24, sources)
    assert np.array_equal(ep, ref.endpoints) and np.array_equal(ln, ref.lengths)


def test_alias_walks_estimate_plain_ppr():
    """Alias walks estimate the plain PPR (binomial z-check of every pair
    with enough expected walks) with the geometric length law."""
    from scipy.stats import chisquare

    import synth
    from exact_ppr import mc_z_check, ppr_exact
    from oracle import oracle as O

    g = synth.chung_lu(150, 900, 2.2, 30, seed=81)
    T = O.alpha_threshold(0.2)
    a = T / 2.0**32
    src = np.array([0, 5, 17, 60, 99], dtype=np.uint32)
    R = 3000
    ep, ln = A.run(g.row_offsets, g.col, g.w, T, 8, R, src)
    pi = ppr_exact(g.n, g.row_offsets, g.col, g.w, a, src)
    dense = np.zeros((len(src), g.n), dtype=np.int64)
    for r in range(len(src)):
        np.add.at(dense[r], ep[r].astype(np.int64), 1)
    ok, info = mc_z_check(dense, pi, R)
    assert ok, info
    L = ln.ravel().astype(np.int64)
    top = 10
    obs = np.array([np.count_nonzero(L == l) for l in range(1, top)] + [np.count_nonzero(L >= top)])
    p = np.array([a * (1 - a) ** (l - 1) for l in range(1, top)] + [(1 - a) ** (top - 1)])
    assert chisquare(obs, p * L.size).pvalue > 1e-4
