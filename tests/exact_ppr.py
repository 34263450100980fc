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


def _spmm(M, X, threads=None):
    """M @ X for a sparse M and a dense X of many columns, the columns split
    over host threads (scipy's product releases the interpreter lock)."""
    import concurrent.futures as cf
    import os

    ns = X.shape[1]
    t = threads or min(16, os.cpu_count() or 1)
    if ns < 16 or t < 2:
        return M @ X
    step = -(-ns // t)
    parts = [np.ascontiguousarray(X[:, i:i + step]) for i in range(0, ns, step)]
    with cf.ThreadPoolExecutor(len(parts)) as ex:
        return np.hstack(list(ex.map(lambda c: M @ c, parts)))


def _series(n, sources, Q, A, dangling, alpha, tol=1e-17, max_iter=100000):
    """pi = sum_k X_k A + alpha (X_k d) e_s, X_{k+1} = X_k Q + (1-alpha)(X_k d) e_s,
    X_0 = e_s. Q, A sparse (continue / absorb), d the dangling indicator."""
    src = np.asarray(sources, dtype=np.int64)
    ns = src.shape[0]
    cols = np.arange(ns)
    # one column per source (nodes x sources); sum_k X_k A = (sum_k X_k) A,
    # so the absorbing part is applied once, to the running sum
    X = np.zeros((n, ns))
    X[src, cols] = 1.0
    Xsum = np.zeros((n, ns))
    back_sum = np.zeros(ns)
    QT = Q.T.tocsr()
    AT = A.T.tocsr()
    for _ in range(max_iter):
        back = dangling @ X  # mass at dangling nodes, returns to the source
        Xsum += X
        back_sum += back
        Xn = _spmm(QT, X)
        Xn[src, cols] += (1.0 - alpha) * back
        X = Xn
        if X.sum() < tol:
            break
    pi = np.ascontiguousarray(_spmm(AT, Xsum).T)
    pi[cols, src] += alpha * back_sum
    return pi


def ppr_exact(n, row_offsets, col, w, alpha, sources):
    P, d = transition(n, row_offsets, col, w)
    return _series(n, sources, (1.0 - alpha) * P, alpha * P, d, alpha)


def chain_exact(n, row_offsets, col, w, alpha, sources, small_nodes, pool_entries, K):
    """Pool-conditioned chain. small_nodes: ids in increasing order; pool_entries
    uint64[len(small_nodes)*K] encoded end | steps<<32 | mark<<48 (mark 1 = stop)."""
    P, d = transition(n, row_offsets, col, w)
    small = np.asarray(small_nodes, dtype=np.int64)
    keep = np.ones(n, dtype=bool)
    keep[small] = False
    Pc = P.tocoo()
    m = keep[Pc.row]  # rows of nodes that are not small keep their edges
    ent = np.asarray(pool_entries, dtype=np.uint64).reshape(small.shape[0], K)
    ends = (ent & np.uint64(0xFFFFFFFF)).astype(np.int64).ravel()
    term = ((ent >> np.uint64(48)) & np.uint64(1)).astype(bool).ravel()
    rows = np.repeat(small, K)  # a small node jumps to each of its K entries with weight 1/K
    Q = sp.coo_matrix((np.concatenate([(1.0 - alpha) * Pc.data[m], np.full(int((~term).sum()), 1.0 / K)]),
                       (np.concatenate([Pc.row[m], rows[~term]]), np.concatenate([Pc.col[m], ends[~term]]))),
                      shape=(n, n)).tocsr()  # duplicates add
    A = sp.coo_matrix((np.concatenate([alpha * Pc.data[m], np.full(int(term.sum()), 1.0 / K)]),
                       (np.concatenate([Pc.row[m], rows[term]]), np.concatenate([Pc.col[m], ends[term]]))),
                      shape=(n, n)).tocsr()
    return _series(n, sources, Q, A, d, alpha)


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
