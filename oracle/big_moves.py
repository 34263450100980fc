"""Exact big moves (Sec. 4.2, Algorithm 4; Lemma 2): CPU oracle, test
infrastructure only.

Only the test suite may import this module. It shares nothing with the GPU
library; it reads a CSR graph (row_offsets, col, w) and nothing else.

What it computes, for one small node v: the distribution of the first k
steps of a walk from v (pick an out-neighbour with probability w / W, then
stop there with probability alpha), split into

* terminated outcomes <t, j>: the walk stopped at t after j steps, and
* active outcomes <t, j>: the walk is still going at t after j steps,

expanded frontier by frontier until the paper's stop rule holds. The sets
follow the algorithm's notation: F is the frontier (mass that has just
arrived at a node and not yet tossed its coin), B the accumulated arrivals
(terminated mass = alpha x B), and the final F becomes the active big moves
((1 - alpha) x F).

Readings where the algorithm is silent or ambiguous (each one is stated in
the design notes as well):

1. Outcomes are kept per (end node, length). The algorithm aggregates by end
   node only; splitting by length gives the same distribution over (end,
   mark) and keeps the walk length, which the step counts need. The stop rule
   still counts distinct end nodes in B, as the algorithm does.
2. A frontier entry at a node without out-neighbours is frozen: it leaves the
   expansion as an active outcome of its own length (the restart to the main
   walk's head cannot be expanded here, since the head is not v). Without it
   that mass would vanish and Lemma 2's sum would fall below 1. Frozen
   entries count towards the stop rule's |F|, and they are still arrivals in
   B (their terminated share is alpha x their mass, like any other arrival).
3. The stop rule is evaluated per node: expand while |B| + |F| < d and the
   previous expansion reached a new end node (|B| grew); the first check
   always passes the second half (prevBSize starts at 0).
4. The frontier is aggregated by node before it is expanded (a node's
   arrival mass is one entry, however many paths reached it).
5. Integer form: probabilities are 62-bit fixed point (units of 2^-62) with a
   floor after every product: an edge e = (u, t) of weight w_e turns the
   continue mass c = floor(a * C / 2^32) of a frontier entry (u, a) into
   floor(c * w_e / W(u)), where C = 2^32 - T and T the walk's coin threshold
   (alpha = T / 2^32 exactly). The first step is floor(w_e * 2^62 / W(v)).
   Terminated weight = floor(a * T / 2^32), active = floor(a * C / 2^32).
   Sums are exact integers, so the result does not depend on the order in
   which edges or entries are visited. Entries of weight 0 are dropped (a
   pick by the first prefix above a draw can never land on them).
6. Table order: entries sorted by their encoding end | steps << 32 |
   mark << 48 (mark 1 = terminated), the same encoding as a pool entry.

A move at a small node then takes one entry of the node's table with
probability weight / (sum of weights): the draw X = floor(D * Wb / 2^64) of a
64-bit uniform D, and the first entry whose inclusive weight prefix exceeds
X, as for an ordinary edge pick (Sec. 3.1).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

ONE = 1 << 62
TERM = 1  # mark of a terminated outcome, as in a pool entry


def _row(row_offsets, col, w, u):
    a, b = int(row_offsets[u]), int(row_offsets[u + 1])
    return [int(x) for x in col[a:b]], [int(x) for x in w[a:b]]


def _expand(row_offsets, col, w, v, d, fixed_k, first, step, max_entries=None):
    """Algorithm 4 for one node, generic over the arithmetic: `first(w_e, W)`
    gives a first-step mass, `step(a, w_e, W)` the mass an edge carries out
    of a frontier entry of mass a. Returns (arrivals B by (t, j), final
    frontier F by t, its length, frozen entries by (t, j)).

    max_entries (optional): a level is expanded only if the table could not
    exceed that many entries afterwards, bounding it by the current entries
    plus two per out-edge of the frontier (one arrival and one frontier
    entry each)."""
    nb, wt = _row(row_offsets, col, w, v)
    if not nb:
        raise ValueError("a big move needs a node with out-neighbours")
    Wv = sum(wt)
    F = {}
    for t, we in zip(nb, wt):
        F[t] = F.get(t, 0) + first(we, Wv)
    j = 1
    B = {(t, 1): a for t, a in F.items()}
    Bt = set(F)
    Z = {}
    prev = 0
    while True:
        if fixed_k is not None:
            if j >= fixed_k:
                break
        elif not (len(Bt) + len(F) + len(Z) < d and prev < len(Bt)):
            break
        if max_entries is not None:
            out_edges = sum(int(row_offsets[u + 1]) - int(row_offsets[u]) for u in F)
            if len(B) + len(F) + len(Z) + 2 * out_edges > max_entries:
                break
        prev = len(Bt)
        nxt = {}
        for u, a in F.items():
            nu, wu = _row(row_offsets, col, w, u)
            if not nu:
                Z[(u, j)] = Z.get((u, j), 0) + a
                continue
            Wu = sum(wu)
            for t, we in zip(nu, wu):
                nxt[t] = nxt.get(t, 0) + step(a, we, Wu)
        j += 1
        for t, a in nxt.items():
            B[(t, j)] = B.get((t, j), 0) + a
            Bt.add(t)
        F = nxt
    return B, F, j, Z


def big_moves_exact(row_offsets, col, w, v, alpha, d, fixed_k=None, max_entries=None):
    """Exact rational big moves of v: {(end, steps, mark): Fraction}. alpha
    is taken as a Fraction; fixed_k replaces the stop rule by exactly fixed_k
    expansion levels (a pool's fixed walk length); max_entries adds the
    size look-ahead of `_expand`."""
    al = Fraction(alpha)
    B, F, k, Z = _expand(row_offsets, col, w, v, d, fixed_k,
                         lambda we, W: Fraction(we, W),
                         lambda a, we, W: a * (1 - al) * Fraction(we, W), max_entries)
    out = {}
    for (t, j), a in B.items():
        out[(t, j, TERM)] = out.get((t, j, TERM), 0) + al * a
    for t, a in F.items():
        out[(t, k, 0)] = out.get((t, k, 0), 0) + (1 - al) * a
    for (t, j), a in Z.items():
        out[(t, j, 0)] = out.get((t, j, 0), 0) + (1 - al) * a
    return {key: p for key, p in out.items() if p != 0}


def big_moves_fixed(row_offsets, col, w, v, T, d, fixed_k=None, max_entries=None):
    """62-bit fixed-point big moves of v for the coin threshold T (alpha =
    T / 2^32): {(end, steps, mark): integer weight}, weights in units of
    2^-62, zero weights dropped."""
    C = (1 << 32) - T
    B, F, k, Z = _expand(row_offsets, col, w, v, d, fixed_k,
                         lambda we, W: (we * ONE) // W,
                         lambda a, we, W: (((a * C) >> 32) * we) // W, max_entries)
    out = {}
    for (t, j), a in B.items():
        key = (t, j, TERM)
        out[key] = out.get(key, 0) + ((a * T) >> 32)
    for t, a in F.items():
        out[(t, k, 0)] = out.get((t, k, 0), 0) + ((a * C) >> 32)
    for (t, j), a in Z.items():
        out[(t, j, 0)] = out.get((t, j, 0), 0) + ((a * C) >> 32)
    return {key: q for key, q in out.items() if q != 0}


def encode(t, steps, mark):
    return int(t) | (int(steps) << 32) | (int(mark) << 48)


def table(row_offsets, col, w, small_nodes, T, d, max_entries=None):
    """Big-move tables of every node in small_nodes (increasing ids): CSR
    offsets u64[len+1], entry encodings u64[], weights u64[] (each node's
    entries in increasing encoding order)."""
    offs = [0]
    ent, wts = [], []
    for v in small_nodes:
        bm = big_moves_fixed(row_offsets, col, w, int(v), T, d, max_entries=max_entries)
        for key in sorted(bm, key=lambda k: encode(*k)):
            ent.append(encode(*key))
            wts.append(bm[key])
        offs.append(len(ent))
    return (np.array(offs, dtype=np.uint64), np.array(ent, dtype=np.uint64),
            np.array(wts, dtype=np.uint64))


def pick(entries, weights, D):
    """One big move from a node's table for the 64-bit uniform D: the first
    entry whose inclusive weight prefix exceeds floor(D * Wb / 2^64)."""
    total = sum(int(q) for q in weights)
    X = (int(D) * total) >> 64
    acc = 0
    for e, q in zip(entries, weights):
        acc += int(q)
        if acc > X:
            return int(e)
    raise AssertionError("draw past the table's total")


# --------------------------------------------------------------------------
# walks that take big moves (small cases; pure Python)
# --------------------------------------------------------------------------
MOVE_CAP = 65536


def tables_by_node(row_offsets, col, w, S, T, d, max_entries=None):
    """{v: (entries, weights)} for every node with 1 <= out-degree <= S."""
    deg = np.diff(np.asarray(row_offsets, dtype=np.int64))
    small = np.flatnonzero((deg >= 1) & (deg <= S))
    offs, ent, wts = table(row_offsets, col, w, small, T, d, max_entries)
    return {int(v): (ent[offs[r]:offs[r + 1]].tolist(), wts[offs[r]:offs[r + 1]].tolist())
            for r, v in enumerate(small)}


def walk(graph, tables, T, seed, s, i):
    """One walk from s (walk id i) under the walk rules of Sec. 2.1: a move
    at a node in `tables` takes one big move (terminated: the walk ends at
    its end node; active: it continues from there), a move at a node without
    out-neighbours returns to s and tosses the coin, any other move picks an
    out-edge by weight and tosses the coin. The draws are those of a plain
    walk: Philox4x32-10 on the counter (i, move, s, 0), x0 and x1 the 64-bit
    draw of a pick, x2 the coin (stop iff x2 < T). Returns (end node, steps,
    moves)."""
    from oracle import oracle as O

    off, col = graph.row_offsets, graph.col
    prefix = graph.prefix()
    key = (seed & 0xFFFFFFFF, seed >> 32)
    tail, steps, m = s, 0, 0
    while True:
        x = [int(a) for a in O.philox4x32_10((i, m, s, 0), key)]
        a, b = int(off[tail]), int(off[tail + 1])
        if a == b:
            tail = s
            steps += 1
            stop = x[2] < T
        elif tail in tables:
            ent, wts = tables[tail]
            e = pick(ent, wts, (x[1] << 32) | x[0])
            tail = e & 0xFFFFFFFF
            steps += (e >> 32) & 0xFFFF
            stop = (e >> 48) & 1 == TERM
        else:
            tail = int(col[a + O.pick(prefix[a:b], x[0], x[1])])
            steps += 1
            stop = x[2] < T
        m += 1
        if not stop and m == MOVE_CAP:
            stop = True
        if stop:
            return tail, steps, m


def run(graph, tables, T, seed, R, sources):
    """Endpoints and step counts [len(sources), R] of walks i = 0..R-1 from
    every source."""
    ep = np.zeros((len(sources), R), dtype=np.uint32)
    ln = np.zeros((len(sources), R), dtype=np.uint32)
    for r, s in enumerate(sources):
        for i in range(R):
            ep[r, i], ln[r, i], _ = walk(graph, tables, T, seed, int(s), i)
    return ep, ln


class LazyBigMoves(dict):
    """Big-move tables (sorted entries, weights) of the small nodes a walk
    visits, built on first use with the fixed-point rules and the size cap."""

    def __init__(self, row_offsets, col, w, T, d, max_entries):
        super().__init__()
        self.args = (row_offsets, col, w)
        self.T, self.d, self.cap = T, d, max_entries

    def __missing__(self, v):
        bm = big_moves_fixed(*self.args, int(v), self.T, self.d, max_entries=self.cap)
        keys = sorted(bm, key=lambda k: encode(*k))
        t = ([encode(*k) for k in keys], [bm[k] for k in keys])
        self[v] = t
        return t


def walk_with_alias(row_offsets, col, w, S, bm_tables, alias_tables, T, seed, s, i):
    """One walk of the paper's design (Algorithm 2 with Sec. 2.2's alias
    picks and Sec. 4.2's big moves): at a node with 1 <= out-degree <= S the
    move takes one big move of its table (pick over the weights with the
    move's 64-bit draw (x1:x0); a terminated entry ends the walk there, an
    active one continues from its end); at any other node with out-edges the
    move takes alias_pick with the same draw and then tosses the coin
    x2 < T; a node without out-edges sends the walk to s and tosses the
    coin. Draws: Philox4x32-10 on (i, move, s, 0). Returns (end, steps)."""
    from oracle import alias as A
    from oracle import oracle as O

    key = (seed & 0xFFFFFFFF, seed >> 32)
    tail, steps, m = s, 0, 0
    while True:
        x = [int(a) for a in O.philox4x32_10((i, m, s, 0), key)]
        D = (x[1] << 32) | x[0]
        a, b = int(row_offsets[tail]), int(row_offsets[tail + 1])
        if a == b:
            tail = s
            steps += 1
            stop = x[2] < T
        elif b - a <= S:
            ent, wts = bm_tables[tail]
            e = pick(ent, wts, D)
            tail = e & 0xFFFFFFFF
            steps += (e >> 32) & 0xFFFF
            stop = (e >> 48) & 1 == TERM
        else:
            P, al, W = alias_tables[tail]
            tail = int(col[a + A.alias_pick(P, al, W, D)])
            steps += 1
            stop = x[2] < T
        m += 1
        if not stop and m == MOVE_CAP:
            stop = True
        if stop:
            return tail, steps


def run_with_alias(row_offsets, col, w, S, d, cap, T, seed, R, sources):
    """Endpoints and steps [len(sources), R] of walk_with_alias."""
    from oracle import alias as A

    bm = LazyBigMoves(row_offsets, col, w, T, d, cap)
    al = A.LazyTables(row_offsets, w)
    ep = np.zeros((len(sources), R), dtype=np.uint32)
    ln = np.zeros((len(sources), R), dtype=np.uint32)
    for r, s in enumerate(sources):
        for i in range(R):
            ep[r, i], ln[r, i] = walk_with_alias(row_offsets, col, w, S, bm, al, T, seed, int(s), i)
    return ep, ln
