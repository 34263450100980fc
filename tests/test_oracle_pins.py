"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test would fail under a plausible mistake in the oracle: a wrong Philox
round or key schedule (KAT, rocRAND), a coin taken before the step or with
the wrong comparison (closed forms F1, F2, length law), a wrong edge pick or
transposed prefix (boundary enumeration, star F3, power iteration), a wrong
restart target (F2, power iteration), a pool that drops or misplaces the
termination mark (Example 5, Lemma 2, pool-conditioned chain), a wrong
aggregation (invariants, brute-force top-k).
"""
import json
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import synth
from oracle import oracle as O
from exact_ppr import chain_exact, dense_counts, mc_z_check, ppr_exact, ppr_networkx

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def graph_from_edges(n, edges, weights=None):
    src = np.array([e[0] for e in edges], dtype=np.uint32)
    dst = np.array([e[1] for e in edges], dtype=np.uint32)
    w = np.ones(len(edges), dtype=np.uint32) if weights is None else np.array(weights, np.uint32)
    return synth.csr_from_edges(n, src, dst, w)


def oracle_graph(g):
    return O.Graph(g.n, g.row_offsets, g.col, g.w)


def T_eff(alpha):
    return O.alpha_threshold(alpha) / 2.0**32


# --------------------------------------------------------------------------
# Philox4x32-10
# --------------------------------------------------------------------------
def test_philox_known_answers():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    assert len(rows) == 3
    for r in rows:
        out = O.philox4x32_10(r[0:4], r[4:6])
        assert [int(x) for x in out] == r[6:10]


ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned k0, k1, c0, c1, c2, c3;
  while (scanf("%x %x %x %x %x %x", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
    rocrand_state_philox4x32_10 st;
    unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
    unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
    unsigned long long off = (((unsigned long long)c1 << 32) | c0) * 4ull;
    rocrand_init(seed, sub, off, &st);
    uint4 v = rocrand4(&st);
    printf("%08x %08x %08x %08x\n", v.x, v.y, v.z, v.w);
  }
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_host():
    """rocRAND's Philox4x32-10 (its header compiled for the host) on random
    keys and counters: seed = key, subsequence = counter words 2-3,
    offset/4 = counter words 0-1 (word 1 kept below 2^30 so the offset fits
    in 64 bits)."""
    rng = np.random.default_rng(7)
    vals = rng.integers(0, 2**32, size=(300, 6), dtype=np.uint64)
    vals[:, 3] %= 2**30  # the offset argument counts 32-bit outputs in 64 bits
    vals[:100, 3] = 0
    vals[:50, 1] = 0
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "p.cpp")
        exe = os.path.join(d, "p")
        with open(src, "w") as f:
            f.write(ROCRAND_PROBE)
        subprocess.check_call(["hipcc", "-O1", src, "-o", exe], stdout=subprocess.DEVNULL,
                              stderr=subprocess.DEVNULL)
        inp = "\n".join(" ".join("%x" % int(x) for x in row) for row in vals) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    got = [[int(x, 16) for x in line.split()] for line in out.strip().splitlines()]
    assert len(got) == len(vals)
    for row, ref in zip(vals, got):
        k = [int(row[0]), int(row[1])]
        c = [int(x) for x in row[2:6]]
        assert [int(x) for x in O.philox4x32_10(c, k)] == ref


# --------------------------------------------------------------------------
# coin threshold and weighted pick
# --------------------------------------------------------------------------
def test_alpha_threshold_values():
    assert O.alpha_threshold(0.1) == 429496730
    assert O.alpha_threshold(0.15) == 644245094
    assert O.alpha_threshold(0.2) == 858993459
    assert O.alpha_threshold(0.5) == 2**31
    assert O.alpha_threshold(1e-12) == 1
    assert O.alpha_threshold(1 - 1e-12) == 2**32 - 1
    for bad in (0.0, 1.0, -0.1, 1.5, float("nan")):
        assert O.alpha_threshold(bad) == 0


def _ceil_div(a, b):
    return -((-a) // b)


def test_pick_boundaries_match_exact_counts():
    """Edge j is chosen for exactly the 64-bit draws r in
    [ceil(P_{j-1} 2^64 / W), ceil(P_j 2^64 / W)): check the pick on both sides
    of every boundary (the pick is monotone in r, so this fixes it)."""
    rng = np.random.default_rng(3)
    rows = [[1], [5], [1, 1], [3, 1, 4, 1, 5, 9, 2, 6], list(rng.integers(1, 1000, 37)),
            [2**32 - 1] * 5, list(rng.integers(1, 2**32 - 1, 12))]
    for w in rows:
        P = np.cumsum(np.array(w, dtype=np.uint64)).astype(np.uint64)
        W = int(P[-1])
        prev = 0
        for j in range(len(w)):
            lo = _ceil_div(prev * 2**64, W)
            hi = _ceil_div(int(P[j]) * 2**64, W)
            assert hi > lo
            for r in (lo, hi - 1, (lo + hi) // 2):
                assert O.pick(P, r & 0xFFFFFFFF, r >> 32) == j
            prev = int(P[j])
        assert hi == 2**64 or hi > 2**64 - 1


# --------------------------------------------------------------------------
# closed forms
# --------------------------------------------------------------------------
def test_cycle_closed_form():
    """F1: directed n-cycle, pi(s, s+k) = alpha (1-alpha)^(k-1) / (1-(1-alpha)^n)."""
    n, alpha, R = 7, 0.2, 200_000
    g = graph_from_edges(n, [(i, (i + 1) % n) for i in range(n)], [3] * n)
    res = O.run(oracle_graph(g), alpha, R, seed=11, sources=[0, 3], topk=0)
    a = T_eff(alpha)
    for row, s in enumerate([0, 3]):
        dense = dense_counts(res.counts[row:row + 1], res.n_distinct[row:row + 1], n)[0]
        pi = np.zeros(n)
        for k in range(1, n + 1):
            pi[(s + k) % n] = a * (1 - a) ** (k - 1) / (1 - (1 - a) ** n)
        ok, info = mc_z_check(dense[None], pi[None], R)
        assert ok, info


def test_dangling_closed_form():
    """F2: s -> t with t dangling: pi(s,t) = 1/(2-alpha), pi(s,s) = (1-alpha)/(2-alpha);
    from t itself every walk ends at t."""
    alpha, R = 0.3, 200_000
    g = graph_from_edges(2, [(0, 1)], [17])
    res = O.run(oracle_graph(g), alpha, R, seed=5, sources=[0, 1], topk=2, want_lengths=True)
    a = T_eff(alpha)
    dense = dense_counts(res.counts, res.n_distinct, 2)
    ok, info = mc_z_check(dense[:1], np.array([[(1 - a) / (2 - a), 1 / (2 - a)]]), R)
    assert ok, info
    assert dense[1, 1] == R and dense[1, 0] == 0
    # a walk always takes at least one step (Ex. 1): no zero lengths
    assert res.lengths.min() >= 1


def test_star_of_self_loops_is_exact_routing():
    """F3: s -> a_i with weights w_i, each a_i with only a self-loop: the walk
    ends at a_i with probability r(s, a_i) = w_i / W, whatever alpha is."""
    w = [1, 2, 3, 10, 50, 7]
    k = len(w)
    edges = [(0, i + 1) for i in range(k)] + [(i + 1, i + 1) for i in range(k)]
    g = graph_from_edges(k + 1, edges, w + [1] * k)
    R = 300_000
    res = O.run(oracle_graph(g), 0.4, R, seed=9, sources=[0], topk=0)
    dense = dense_counts(res.counts, res.n_distinct, k + 1)[0]
    pi = np.array([0.0] + [x / sum(w) for x in w])
    ok, info = mc_z_check(dense[None], pi[None], R)
    assert ok, info


def test_length_is_geometric():
    """F4: the number of steps of a plain walk is Geometric(alpha) on {1,2,...}
    for any graph (Sec. 2.1: expected length 1/alpha; Lemma 2 proof)."""
    g = synth.small_graph()
    alpha = 0.2
    res = O.run(oracle_graph(g), alpha, 200, seed=21, topk=0, want_lengths=True,
                want_counts=False)
    L = res.lengths.ravel().astype(np.int64)
    a = T_eff(alpha)
    N = L.size
    assert L.min() >= 1
    kmax = 30
    obs = np.bincount(np.minimum(L, kmax), minlength=kmax + 1)[1:]
    exp = np.array([a * (1 - a) ** (k - 1) for k in range(1, kmax)] + [(1 - a) ** (kmax - 1)]) * N
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    from scipy.stats import chi2 as chi2d
    assert chi2d.sf(chi2, kmax - 1) > 1e-4, chi2
    assert res.stats["steps"] == L.sum() == res.stats["moves"]
    # mean length within 6 sigma of 1/alpha
    sd = math.sqrt((1 - a) / a**2 / N)
    assert abs(L.mean() - 1 / a) < 6 * sd


def test_move_cap():
    """With the smallest threshold (T = 1: a move stops only on x2 == 0,
    probability 2^-32) both walks on a directed 3-cycle run to the cap of
    65,536 moves and stop there, at the current tail: node 65536 mod 3 = 1
    of the cycle 0 -> 1 -> 2 -> 0. A cap one move shorter or longer, or a
    cap that is never applied, fails one of these."""
    g = graph_from_edges(3, [(0, 1), (1, 2), (2, 0)])
    res = O.run(oracle_graph(g), 1e-12, 2, seed=1, sources=[0], topk=1, want_lengths=True)
    assert O.MOVE_CAP == 65536
    assert res.stats["capped"] == 2 and res.stats["walks"] == 2
    assert np.array_equal(res.lengths.ravel(), [O.MOVE_CAP, O.MOVE_CAP])
    assert res.stats["moves"] == res.stats["steps"] == 2 * O.MOVE_CAP
    assert res.counts[0][0].tolist() == [O.MOVE_CAP % 3, 2]  # (node, count): both walks end at node 1


# --------------------------------------------------------------------------
# whole-method checks against FP64 PageRank
# --------------------------------------------------------------------------
def test_exact_reference_matches_networkx():
    """Pins the FP64 series against networkx PageRank (restart form)."""
    g = graph_from_edges(6, [(0, 1), (0, 2), (0, 2), (1, 3), (2, 3), (3, 0), (3, 4), (4, 4),
                             (2, 5)], [1, 2, 3, 4, 5, 6, 7, 8, 9])
    for s in (0, 4, 5):
        a = 0.15
        ref = ppr_exact(g.n, g.row_offsets, g.col, g.w, a, [s])[0]
        nxv = ppr_networkx(g.n, g.row_offsets, g.col, g.w, a, s)
        assert np.allclose(ref, nxv, atol=1e-9), (s, ref, nxv)
        assert abs(ref.sum() - 1) < 1e-12


@pytest.mark.parametrize("seed", [1, 2])
def test_plain_walks_match_power_iteration(seed):
    """S0 on the 2,000-node Chung-Lu graph: counts within the binomial
    3-sigma bound of the FP64 PPR for 40 sources."""
    g = synth.small_graph()
    alpha, R = 0.2, 20_000
    rng = np.random.default_rng(seed)
    deg = g.degrees()
    src = np.unique(np.concatenate([rng.choice(g.n, 36, replace=False),
                                    np.flatnonzero(deg == 0)[:2], [int(np.argmax(deg))]]))
    res = O.run(oracle_graph(g), alpha, R, seed=seed, sources=src, topk=0)
    pi = ppr_exact(g.n, g.row_offsets, g.col, g.w, T_eff(alpha), src)
    ok, info = mc_z_check(dense_counts(res.counts, res.n_distinct, g.n), pi, R)
    assert ok, info


def test_guarantee_of_definition_1():
    """Definition 1: with omega = (2 + 2 eps/3) ln(2/p_f) / (eps^2 delta) walks,
    pairs with pi >= delta have relative error <= eps except with probability
    p_f."""
    g = synth.chung_lu(300, 2400, 2.2, 20, seed=77)
    eps, delta, pf = 0.2, 0.05, 0.01
    R = math.ceil((2 + 2 * eps / 3) * math.log(2 / pf) / (eps**2 * delta))
    alpha = 0.25
    src = np.arange(0, 300, 3)
    res = O.run(oracle_graph(g), alpha, R, seed=3, sources=src, topk=0)
    pi = ppr_exact(g.n, g.row_offsets, g.col, g.w, T_eff(alpha), src)
    est = dense_counts(res.counts, res.n_distinct, g.n) / R
    sel = pi >= delta
    bad = np.abs(est[sel] - pi[sel]) > eps * pi[sel]
    assert sel.sum() > 50
    assert bad.mean() <= pf


# --------------------------------------------------------------------------
# short-walk pool (big moves)
# --------------------------------------------------------------------------
def test_example5_pool_distribution():
    """Example 5: on v2->v3->v4->v3 with alpha = 0.5 and 3 steps, the pool
    walks of v2 follow the big-move distribution printed in the paper."""
    fx = json.load(open(os.path.join(GOLDEN, "example5_big_moves.json")))
    n = 5
    g = graph_from_edges(n, [tuple(e) for e in fx["edges"]] + [(0, 1), (1, 0)])
    K = 1 << 16
    G = oracle_graph(g)
    pool = O.Pool(G, S=4, L=fx["steps"], K=K, alpha=fx["alpha"], seed=123)
    deg = g.degrees()
    small = np.flatnonzero((deg >= 1) & (deg <= 4))
    r = int(np.flatnonzero(small == fx["source"])[0])
    ent = pool.entries().reshape(len(small), K)[r]
    end = (ent & np.uint64(0xFFFFFFFF)).astype(np.int64)
    steps = ((ent >> np.uint64(32)) & np.uint64(0xFFFF)).astype(np.int64)
    term = ((ent >> np.uint64(48)) & np.uint64(1)).astype(bool)
    # coarse: the paper's three big moves
    obs = [np.count_nonzero((end == bm["end"]) & (term == bm["terminated"]))
           for bm in fx["big_moves"]]
    assert sum(obs) == K
    exp = [bm["p"] * K for bm in fx["big_moves"]]
    from scipy.stats import chisquare
    assert chisquare(obs, exp).pvalue > 1e-4
    # fine: by length
    obs2 = [np.count_nonzero((end == e) & (steps == L) & (term == t))
            for e, L, t, _ in fx["derived_by_length"]["entries"]]
    assert sum(obs2) == K
    assert chisquare(obs2, [p * K for *_, p in fx["derived_by_length"]["entries"]]).pvalue > 1e-4


def test_lemma2_pool_masses():
    """Lemma 2: on a graph without dangling nodes the terminated mass of an
    L-step expansion is 1-(1-alpha)^L and the active mass (1-alpha)^L; every
    active entry has exactly L steps."""
    n = 400
    rng = np.random.default_rng(4)
    edges = [(u, int(v)) for u in range(n) for v in rng.integers(0, n, 3)]
    g = graph_from_edges(n, edges, rng.integers(1, 9, len(edges)))
    alpha, L, K = 0.3, 3, 256
    pool = O.Pool(oracle_graph(g), S=8, L=L, K=K, alpha=alpha, seed=5)
    ent = pool.entries()
    term = ((ent >> np.uint64(48)) & np.uint64(1)).astype(bool)
    steps = ((ent >> np.uint64(32)) & np.uint64(0xFFFF)).astype(np.int64)
    a = T_eff(alpha)
    p_act = (1 - a) ** L
    N = ent.size
    sd = math.sqrt(p_act * (1 - p_act) / N)
    assert abs((~term).mean() - p_act) < 6 * sd
    assert np.all(steps[~term] == L)
    assert steps.min() >= 1 and steps.max() <= L


def test_pool_stops_at_dangling_nodes():
    """A pool walk that reaches a node without out-neighbours stops there,
    still active, so the main walk restarts to its own head on its next move."""
    g = graph_from_edges(3, [(0, 1), (1, 2)])
    pool = O.Pool(oracle_graph(g), S=4, L=3, K=1024, alpha=0.5, seed=8)
    ent = pool.entries().reshape(2, 1024)  # small nodes 0 and 1
    for r, v in enumerate((0, 1)):
        end = (ent[r] & np.uint64(0xFFFFFFFF)).astype(np.int64)
        term = ((ent[r] >> np.uint64(48)) & np.uint64(1)).astype(bool)
        steps = ((ent[r] >> np.uint64(32)) & np.uint64(0xFFFF)).astype(np.int64)
        assert np.all(end[~term] == 2)  # active entries end at the dangling node
        if v == 0:
            assert set(steps[~term]) <= {2}
            assert set(np.unique(end)) <= {1, 2}


@pytest.mark.parametrize("K", [8, 64])
def test_stitched_walks_match_pool_conditioned_chain(K):
    """S1: given the pool, walks follow the chain in which small nodes jump by
    a uniformly chosen pool entry; FP64 solution of that chain, 3-sigma."""
    g = synth.small_graph()
    alpha, R, S, L = 0.2, 20_000, 8, 3
    G = oracle_graph(g)
    pool = O.Pool(G, S=S, L=L, K=K, alpha=alpha, seed=17)
    deg = g.degrees()
    small = np.flatnonzero((deg >= 1) & (deg <= S))
    rng = np.random.default_rng(K)
    src = np.unique(np.concatenate([rng.choice(g.n, 30, replace=False), small[:5],
                                    np.flatnonzero(deg == 0)[:2]]))
    res = O.run(G, alpha, R, seed=4, sources=src, topk=0, pool=pool)
    pi = chain_exact(g.n, g.row_offsets, g.col, g.w, T_eff(alpha), src, small, pool.entries(), K)
    ok, info = mc_z_check(dense_counts(res.counts, res.n_distinct, g.n), pi, R)
    assert ok, info
    assert res.stats["stitched_moves"] > 0
    assert res.stats["steps"] > res.stats["moves"]


def test_pool_bias_shrinks_with_K():
    """The pool-conditioned PPR approaches the true PPR as K grows."""
    g = synth.chung_lu(200, 1200, 2.2, 50, seed=31)
    alpha, S, L = 0.2, 6, 3
    G = oracle_graph(g)
    deg = g.degrees()
    small = np.flatnonzero((deg >= 1) & (deg <= S))
    src = np.arange(0, 200, 5)
    a = T_eff(alpha)
    truth = ppr_exact(g.n, g.row_offsets, g.col, g.w, a, src)
    err = {}
    for K in (8, 512):
        e = []
        for seed in (1, 2, 3):
            pool = O.Pool(G, S=S, L=L, K=K, alpha=alpha, seed=seed)
            pi = chain_exact(g.n, g.row_offsets, g.col, g.w, a, src, small, pool.entries(), K)
            e.append(np.abs(pi - truth).sum(axis=1).mean())
        err[K] = float(np.mean(e))
    assert err[512] < 0.5 * err[8], err


# --------------------------------------------------------------------------
# invariants of the aggregation
# --------------------------------------------------------------------------
def _reachable(g, s):
    off = g.row_offsets.astype(np.int64)
    seen = {s}
    stack = [s]
    while stack:
        u = stack.pop()
        nb = g.col[off[u]:off[u + 1]].tolist() if off[u + 1] > off[u] else [s]
        for v in nb:
            if v not in seen:
                seen.add(v)
                stack.append(v)
    return seen


def test_invariants_counts_topk_digest():
    g = synth.small_graph()
    G = oracle_graph(g)
    R, k = 100, 16
    src = np.arange(0, g.n, 7, dtype=np.uint32)
    res = O.run(G, 0.2, R, seed=1, sources=src, topk=k, want_endpoints=True)
    for row, s in enumerate(src.tolist()):
        nd = int(res.n_distinct[row])
        c = res.counts[row]
        # I1: counts sum to R; sorted by t; zero padding after n_distinct
        assert int(c[:nd, 1].sum()) == R
        assert np.all(np.diff(c[:nd, 0].astype(np.int64)) > 0)
        assert np.all(c[nd:] == 0)
        # counts agree with the raw endpoints
        t, cnt = np.unique(res.endpoints[row], return_counts=True)
        assert np.array_equal(t, c[:nd, 0]) and np.array_equal(cnt, c[:nd, 1])
        # I2: every endpoint reachable from s (dangling nodes lead back to s)
        reach = _reachable(g, s)
        assert set(t.tolist()) <= reach
        # I6: top-k is the prefix of the counts sorted by (count desc, id asc)
        order = sorted(zip(c[:nd, 1].tolist(), c[:nd, 0].tolist()), key=lambda x: (-x[0], x[1]))
        want = [(tt, cc) for cc, tt in order[:k]] + [(0xFFFFFFFF, 0)] * max(0, k - nd)
        assert [tuple(x) for x in res.topk[row].tolist()] == want
        # digest
        d = sum(O.digest_term(s, int(tt), int(cc)) for tt, cc in c[:nd]) % 2**64
        assert int(res.digest[row]) == d


def test_thread_count_and_subset_invariance():
    """I4/I7: results depend only on (graph, params, seed, source), not on the
    thread count or on which other sources run alongside."""
    g = synth.small_graph()
    G = oracle_graph(g)
    full = O.run(G, 0.2, 50, seed=9, topk=8, nthreads=1)
    par = O.run(G, 0.2, 50, seed=9, topk=8, nthreads=8)
    assert np.array_equal(full.counts, par.counts) and np.array_equal(full.topk, par.topk)
    assert full.stats == par.stats
    sub = np.array([5, 1999, 17, 17, 0], dtype=np.uint32)
    part = O.run(G, 0.2, 50, seed=9, sources=sub, topk=8)
    for row, s in enumerate(sub):
        assert np.array_equal(part.counts[row], full.counts[s])
        assert np.array_equal(part.topk[row], full.topk[s])
        assert part.digest[row] == full.digest[s]


def test_invalid_inputs_rejected():
    off = np.array([0, 1, 1], dtype=np.uint64)
    with pytest.raises(ValueError):
        O.Graph(2, off, np.array([2], np.uint32), np.array([1], np.uint32))  # col >= n
    with pytest.raises(ValueError):
        O.Graph(2, off, np.array([1], np.uint32), np.array([0], np.uint32))  # w = 0
    with pytest.raises(ValueError):
        O.Graph(2, np.array([0, 2, 1], np.uint64), np.array([1], np.uint32),
                np.array([1], np.uint32))
    g = graph_from_edges(2, [(0, 1)])
    with pytest.raises(ValueError):
        O.run(oracle_graph(g), 0.2, 10, 1, sources=[2])
    with pytest.raises(ValueError):
        O.run(oracle_graph(g), 1.0, 10, 1)
