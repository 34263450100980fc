"""FP64 references for the quantity the walks estimate.

* `ppr_exact` — the definition of Sec. 2.1 written as a series: a walk from s
  takes at least one step, after every step stops with probability alpha, and
  a node without out-neighbours sends it back to s:
      pi(s,.) = sum_{k>=1} alpha (1-alpha)^(k-1) e_s P_s^k
  where P_s is the weight-normalised transition matrix with every dangling
  row replaced by e_s.
* `chain_exact` — the same for walks that, at small nodes, take one entry of
  a given short-walk pool (uniform over its K slots; a terminated entry
  absorbs at its end node, an active one continues from there).
* `ppr_networkx` — an independent route through networkx's PageRank, using
  pi = (pi_RWR - alpha e_s) / (1 - alpha), where pi_RWR is random walk with
  restart with restart probability alpha and dangling mass sent to s.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def transition(n, row_offsets, col, w):
    off = np.asarray(row_offsets, dtype=np.int64)
    deg = np.diff(off)
    rows = np.repeat(np.arange(n), deg)
    W = np.zeros(n, dtype=np.float64)
    np.add.at(W, rows, np.asarray(w, dtype=np.float64))
    vals = np.asarray(w, dtype=np.float64) / W[rows]
    P = sp.csr_matrix((vals, (rows, np.asarray(col, dtype=np.int64))), shape=(n, n))
    dangling = (deg == 0).astype(np.float64)
    return P, dangling


def _series(n, sources, Q, A, dangling, alpha, tol=1e-17, max_iter=100000):
    """pi = sum_k X_k A + alpha (X_k d) e_s, X_{k+1} = X_k Q + (1-alpha)(X_k d) e_s,
    X_0 = e_s. Q, A sparse (continue / absorb), d the dangling indicator."""
    src = np.asarray(sources, dtype=np.int64)
    ns = src.shape[0]
    X = np.zeros((ns, n))
    X[np.arange(ns), src] = 1.0
    pi = np.zeros((ns, n))
    QT = Q.T.tocsr()
    AT = A.T.tocsr()
    for _ in range(max_iter):
        back = X @ dangling  # mass at dangling nodes, returns to the source
        pi += (AT @ X.T).T
        pi[np.arange(ns), src] += alpha * back
        Xn = (QT @ X.T).T
        Xn[np.arange(ns), src] += (1.0 - alpha) * back
        X = Xn
        if X.sum() < tol:
            break
    return pi


def ppr_exact(n, row_offsets, col, w, alpha, sources):
    P, d = transition(n, row_offsets, col, w)
    return _series(n, sources, (1.0 - alpha) * P, alpha * P, d, alpha)


def chain_exact(n, row_offsets, col, w, alpha, sources, small_nodes, pool_entries, K):
    """Pool-conditioned chain. small_nodes: ids in increasing order; pool_entries
    uint64[len(small_nodes)*K] encoded end | steps<<32 | mark<<48 (mark 1 = stop)."""
    P, d = transition(n, row_offsets, col, w)
    P = P.tolil()
    Q = ((1.0 - alpha) * P).tolil()
    A = (alpha * P).tolil()
    ent = np.asarray(pool_entries, dtype=np.uint64).reshape(len(small_nodes), K)
    for r, v in enumerate(small_nodes):
        Q.rows[v] = []
        Q.data[v] = []
        A.rows[v] = []
        A.data[v] = []
        ends = (ent[r] & np.uint64(0xFFFFFFFF)).astype(np.int64)
        term = ((ent[r] >> np.uint64(48)) & np.uint64(1)).astype(bool)
        for e, t in zip(ends, term):
            if t:
                A[v, e] = A[v, e] + 1.0 / K
            else:
                Q[v, e] = Q[v, e] + 1.0 / K
    return _series(n, sources, Q.tocsr(), A.tocsr(), d, alpha)


def ppr_networkx(n, row_offsets, col, w, alpha, s):
    import networkx as nx

    G = nx.DiGraph()
    G.add_nodes_from(range(n))
    off = np.asarray(row_offsets, dtype=np.int64)
    for u in range(n):
        for e in range(off[u], off[u + 1]):
            v = int(col[e])
            if G.has_edge(u, v):
                G[u][v]["weight"] += float(w[e])
            else:
                G.add_edge(u, v, weight=float(w[e]))
    rwr = nx.pagerank(G, alpha=1.0 - alpha, personalization={s: 1.0}, dangling={s: 1.0},
                      weight="weight", tol=1e-15, max_iter=100000)
    vec = np.array([rwr[i] for i in range(n)])
    vec[s] -= alpha
    return vec / (1.0 - alpha)


def mc_z_check(counts_dense, pi, R, min_expect=10.0, frac_limit=0.005, zmax=6.0):
    """Binomial 3-sigma acceptance: pairs with R*pi >= min_expect must have
    |z| > 3 for at most frac_limit of them and |z| <= zmax for all; pairs with
    pi == 0 must have count 0. Returns (ok, details)."""
    c = np.asarray(counts_dense, dtype=np.float64)
    zero = pi <= 1e-300
    bad_zero = int(np.count_nonzero(c[zero]))
    sel = (R * pi >= min_expect) & (pi < 1.0)
    mu = R * pi[sel]
    sd = np.sqrt(R * pi[sel] * (1.0 - pi[sel]))
    z = (c[sel] - mu) / sd
    n_sel = int(sel.sum())
    over = int(np.count_nonzero(np.abs(z) > 3.0))
    zm = float(np.max(np.abs(z))) if n_sel else 0.0
    ok = bad_zero == 0 and n_sel > 0 and over <= max(1, math.ceil(frac_limit * n_sel)) and zm <= zmax
    return ok, dict(pairs=n_sel, over3=over, max_abs_z=zm, nonzero_where_pi_zero=bad_zero)


def dense_counts(counts, n_distinct, n):
    """[n_src, R, 2] padded (t, count) -> dense [n_src, n]."""
    ns = counts.shape[0]
    out = np.zeros((ns, n), dtype=np.int64)
    for i in range(ns):
        k = int(n_distinct[i])
        out[i, counts[i, :k, 0].astype(np.int64)] = counts[i, :k, 1]
    return out
