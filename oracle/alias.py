"""Alias tables and alias trees (Sec. 2.2, Algorithm 1, Example 2; Sec. 4.1,
Algorithm 3, Examples 3-4, Lemma 1): CPU oracle, test infrastructure only.

Only the test suite may import this module; it shares nothing with the GPU
library.

Integer form. For n items with integer weights w (all >= 1) and total W,
Algorithm 1's switch probability p(e) = n r(e) is kept as the integer
P(e) = n w(e) in units of 1/W, so "1" is W and every transfer is exact: the
table ends with every P in [0, W] and no item stranded by rounding. Slot i
holds W units: P[i] for item i itself and W - P[i] for alias[i]. Algorithm
1 leaves the order of its transfers free; here the items below W are
filled oldest first by the earliest item still above W (item order), and
an item that falls below W while giving joins the end of the fill order.
Example 2's printed result follows from that order.

A pick maps one 64-bit uniform D to X = floor(D n W / 2^64) in [0, n W):
slot i = X div W (uniform over the n items) and U = X mod W (uniform over
[0, W)); the result is item i if U < P(i), else its alias. Each item e then
owns exactly n w(e) of the n W values of X, so the pick hits e with
probability w(e) / W up to the 2^-64 granularity of D.

Alias tree (Algorithm 3): a set larger than d is split into b = ceil(n / d)
disjoint subsets; a subset's weight is the sum of its items' weights
(integers, no normalisation needed); each subset gets its own alias table,
and the set of subsets is treated the same way, recursively, until a level
has at most d items. The paper splits at random; Lemma 1 holds for any
partition, so the split is a parameter (contiguous blocks of d items in
item order by default, the layout the prefix trees of the hot path use). A
pick descends from the root with one 64-bit draw per level.
"""
from __future__ import annotations


def alias_table(w):
    """Integer alias table (Sec. 2.2, Algorithm 1): returns (P, alias, W)
    with P[i] in [0, W] the units of slot i kept by item i, in units of
    1/W; the rest of the slot goes to alias[i]. One sweep over the donors
    (items above W, in item order): each fills the oldest unfilled slots
    until it is down to W or below; a donor that ends below W becomes a
    slot to fill itself, after all those already waiting."""
    w = [int(x) for x in w]
    if not w or min(w) < 1:
        raise ValueError("alias table needs at least one item, all weights >= 1")
    n, W = len(w), sum(w)
    P = [n * x for x in w]
    alias = list(range(n))
    to_fill = [i for i in range(n) if P[i] < W]  # grows at the end while donors give
    donors = [i for i in range(n) if P[i] > W]
    nxt = 0
    for y in donors:
        while P[y] > W:  # deficits and surpluses balance exactly, so a slot is always waiting
            x = to_fill[nxt]
            nxt += 1
            alias[x] = y
            P[y] -= W - P[x]
        if P[y] < W:
            to_fill.append(y)
    # every item owns exactly n w(e) units over all slots
    own = list(P)
    for i in range(n):
        if alias[i] != i:
            own[alias[i]] += W - P[i]
    assert own == [n * x for x in w] and all(0 <= p <= W for p in P)
    return P, alias, W


def alias_pick(P, alias, W, D):
    """Item chosen by the 64-bit uniform D (see the module header)."""
    n = len(P)
    X = (int(D) * n * W) >> 64
    i, U = divmod(X, W)
    return i if U < P[i] else alias[i]


def contiguous_split(n, d):
    """Blocks of d consecutive items (the last one shorter)."""
    return [list(range(a, min(a + d, n))) for a in range(0, n, d)]


def alias_tree(w, d, split=contiguous_split):
    """Algorithm 3: a list of levels from the leaves up. Level 0 holds the
    items' subsets over the original items; each level is a list of groups
    (members, P, alias, W) whose members index the level below (the items
    for level 0). The last level has one group: the root."""
    if d < 2:
        raise ValueError("the degree threshold must be at least 2")
    weights = [int(x) for x in w]
    levels = []
    while True:
        n = len(weights)
        groups = [list(range(n))] if n <= d else split(n, d)
        assert sorted(i for g in groups for i in g) == list(range(n)), "not a partition"
        level = []
        for g in groups:
            P, al, W = alias_table([weights[i] for i in g])
            level.append((g, P, al, W))
        levels.append(level)
        if len(groups) == 1:
            return levels
        weights = [W for _, _, _, W in level]


def alias_tree_pick(levels, draws):
    """Descend from the root: at each level the group's alias table picks a
    member with the next 64-bit draw; returns the original item index."""
    g = 0
    for depth, level in enumerate(reversed(levels)):
        members, P, al, W = level[g]
        g = members[alias_pick(P, al, W, draws[depth])]
    return g


# --------------------------------------------------------------------------
# walks that pick with alias tables (small cases; pure Python)
# --------------------------------------------------------------------------
MOVE_CAP = 65536


def row_tables(row_offsets, w):
    """{v: (P, alias, W)} for every node with out-edges."""
    out = {}
    for v in range(len(row_offsets) - 1):
        a, b = int(row_offsets[v]), int(row_offsets[v + 1])
        if a < b:
            out[v] = alias_table(w[a:b])
    return out


class LazyTables(dict):
    """Alias tables of the rows a walk visits, built on first use."""

    def __init__(self, row_offsets, w):
        super().__init__()
        self.row_offsets, self.w = row_offsets, w

    def __missing__(self, v):
        a, b = int(self.row_offsets[v]), int(self.row_offsets[v + 1])
        t = alias_table(self.w[a:b])
        self[v] = t
        return t


def walk(row_offsets, col, tables, T, seed, s, i):
    """One walk from s (walk id i) under Sec. 2.1's rules with alias picks:
    move m draws Philox4x32-10 on (i, m, s, 0) with key (seed low, seed
    high); at a node with out-edges the edge is alias_pick(..., (x1:x0)) and
    the walk then stops iff x2 < T; a node without out-edges returns the walk
    to s and tosses the coin; 65,536 moves at most. Returns (end, steps)."""
    from oracle import oracle as O

    key = (seed & 0xFFFFFFFF, seed >> 32)
    tail, steps, m = s, 0, 0
    while True:
        x = [int(a) for a in O.philox4x32_10((i, m, s, 0), key)]
        a, b = int(row_offsets[tail]), int(row_offsets[tail + 1])
        if a == b:
            tail = s
        else:
            P, al, W = tables[tail]
            tail = int(col[a + alias_pick(P, al, W, (x[1] << 32) | x[0])])
        steps += 1
        m += 1
        if x[2] < T or m == MOVE_CAP:
            return tail, steps


def run(row_offsets, col, w, T, seed, R, sources):
    """Endpoints and steps [len(sources), R]."""
    import numpy as np

    tables = LazyTables(row_offsets, w)
    ep = np.zeros((len(sources), R), dtype=np.uint32)
    ln = np.zeros((len(sources), R), dtype=np.uint32)
    for r, s in enumerate(sources):
        for i in range(R):
            ep[r, i], ln[r, i] = walk(row_offsets, col, tables, T, seed, int(s), i)
    return ep, ln
