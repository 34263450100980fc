"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.

This module holds no step of the PageRank method: it only generates graphs
(canonical CSR with uint32 edge weights) and source lists. The paper measures
on SNAP graphs (Table 2, Section 5.1) that are not available here; the
generators below stand in for them with the degree skew of those graphs:

* directed Chung-Lu: expected out-weight of node i proportional to
  (i+1)^(-1/(gamma-1)); in-weights follow the same law under an independent
  seeded permutation; m (src, dst) pairs drawn independently; multi-edges and
  self-loops kept.
* R-MAT (Chakrabarti, Zhan, Faloutsos 2004) with a seeded vertex relabelling.

Weights are uniform integers or a Zipf law clipped to [1, wmax].
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_SRC = os.path.join(_HERE, "csrc", "graphgen.c")
_lib = None


def build(force: bool = True) -> str:
    """Compile the generator library with gcc (host code only)."""
    import subprocess

    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c99", "-fPIC", "-shared", "-pthread",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    lib.gg_permutation.argtypes = [u32, u64, P]
    lib.gg_chung_lu_edges.argtypes = [u32, u64, P, P, P, u32, u32, u64, i32, P, P, P]
    lib.gg_rmat_edges.argtypes = [u32, u64, u32, u32, u32, P, P, u32, u32, u64, i32, P, P, P]
    lib.gg_build_csr.argtypes = [u32, u64, P, P, P, i32, P, P, P]
    lib.gg_build_csr.restype = i32
    _lib = lib
    return lib


def _ptr(a: np.ndarray | None):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


@dataclass
class CSRGraph:
    """Canonical CSR: row_offsets uint64[n+1], col uint32[m], w uint32[m]."""

    n: int
    row_offsets: np.ndarray
    col: np.ndarray
    w: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_offsets).astype(np.int64)


def permutation(n: int, seed: int) -> np.ndarray:
    perm = np.empty(n, dtype=np.uint32)
    _load().gg_permutation(n, seed, _ptr(perm))
    return perm


def csr_from_edges(n: int, src, dst, w, nthreads: int | None = None, meta=None) -> CSRGraph:
    """Canonical CSR (edges sorted by (src, dst, w)) from an edge list."""
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    w = np.ascontiguousarray(w, dtype=np.uint32)
    m = src.shape[0]
    assert dst.shape[0] == m and w.shape[0] == m
    off = np.empty(n + 1, dtype=np.uint64)
    col = np.empty(max(m, 1), dtype=np.uint32)
    wo = np.empty(max(m, 1), dtype=np.uint32)
    rc = _load().gg_build_csr(n, m, _ptr(src), _ptr(dst), _ptr(w),
                              nthreads or default_threads(), _ptr(off), _ptr(col), _ptr(wo))
    if rc != 0:
        raise ValueError("edge endpoint out of range or allocation failure")
    return CSRGraph(n=n, row_offsets=off, col=col[:m], w=wo[:m], meta=dict(meta or {}))


def zipf_clipped_cdf(s: float, wmax: int) -> np.ndarray:
    """CDF over {1..wmax} of Zipf(s) on {1, 2, ...} with values above wmax
    clipped to wmax."""
    from scipy.special import zeta

    k = np.arange(1, wmax, dtype=np.float64)
    z = float(zeta(s, 1))
    pm = np.empty(wmax, dtype=np.float64)
    pm[:-1] = k ** (-s) / z
    pm[-1] = float(zeta(s, wmax)) / z
    cdf = np.cumsum(pm)
    cdf /= cdf[-1]
    return cdf


def _weights(law: str, wmax: int, zipf_s: float | None):
    if law == "uniform":
        return None, 0
    if law == "zipf":
        cdf = zipf_clipped_cdf(float(zipf_s), wmax)
        return cdf, wmax
    raise ValueError(law)


def chung_lu(n: int, m: int, gamma: float, wmax: int, seed: int, weight_law="uniform",
             zipf_s=None, nthreads=None) -> CSRGraph:
    theta = np.arange(1, n + 1, dtype=np.float64) ** (-1.0 / (gamma - 1.0))
    cdf_out = np.cumsum(theta)
    cdf_out /= cdf_out[-1]
    perm = permutation(n, seed ^ 0x5EED)
    theta_in = np.empty(n, dtype=np.float64)
    theta_in[perm] = theta
    cdf_in = np.cumsum(theta_in)
    cdf_in /= cdf_in[-1]
    wcdf, wlen = _weights(weight_law, wmax, zipf_s)
    src = np.empty(m, dtype=np.uint32)
    dst = np.empty(m, dtype=np.uint32)
    w = np.empty(m, dtype=np.uint32)
    nt = nthreads or default_threads()
    _load().gg_chung_lu_edges(n, m, _ptr(cdf_out), _ptr(cdf_in), _ptr(wcdf), wlen, wmax, seed,
                              nt, _ptr(src), _ptr(dst), _ptr(w))
    meta = dict(kind="chung-lu", n=n, m=m, gamma=gamma, wmax=wmax, weight_law=weight_law,
                seed=seed)
    g = csr_from_edges(n, src, dst, w, nt, meta)
    return g


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, wmax: int, seed: int,
         weight_law="zipf", zipf_s=None, permute=True, nthreads=None) -> CSRGraph:
    n = 1 << scale
    m = edge_factor * n
    ta = int(round(a * 2**32))
    tab = int(round((a + b) * 2**32))
    tabc = int(round((a + b + c) * 2**32))
    perm = permutation(n, seed ^ 0xA11CE) if permute else None
    wcdf, wlen = _weights(weight_law, wmax, zipf_s)
    src = np.empty(m, dtype=np.uint32)
    dst = np.empty(m, dtype=np.uint32)
    w = np.empty(m, dtype=np.uint32)
    nt = nthreads or default_threads()
    _load().gg_rmat_edges(scale, m, ta, tab, tabc, _ptr(perm), _ptr(wcdf), wlen, wmax, seed, nt,
                          _ptr(src), _ptr(dst), _ptr(w))
    meta = dict(kind="rmat", scale=scale, n=n, m=m, abcd=(a, b, c, 1 - a - b - c), wmax=wmax,
                weight_law=weight_law, zipf_s=zipf_s, seed=seed, permuted=permute)
    g = csr_from_edges(n, src, dst, w, nt, meta)
    del src, dst, w
    return g


# ---------------------------------------------------------------------------
# The workloads. Seeds are fixed here; both the oracle and the GPU path read
# the same arrays.
# ---------------------------------------------------------------------------

SMALL = dict(name="chung-lu n=2000 m=20000", alpha=0.2, R=100, seed=1, topk=16, stitch=None)
MEDIUM = dict(name="rmat scale 20", alpha=0.15, R=200, seed=2, topk=32, stitch=None)
SCALE24 = dict(name="rmat scale 24", alpha=0.15, R=128, seed=3, topk=32,
               stitch=dict(S=32, L=3, K=64, seed=3), hub_threshold=4096)


def small_graph(nthreads=None) -> CSRGraph:
    """Directed Chung-Lu, 2,000 nodes, 20,000 edges, out-degree exponent 2.1,
    weights uniform in [1, 100]."""
    return chung_lu(2000, 20000, 2.1, 100, seed=1000, weight_law="uniform", nthreads=nthreads)


def medium_graph(nthreads=None) -> CSRGraph:
    """R-MAT scale 20, edge factor 16, (a,b,c,d) = (0.57, 0.19, 0.19, 0.05),
    weights Zipf(1.5) clipped to [1, 1000]."""
    return rmat(20, 16, 0.57, 0.19, 0.19, wmax=1000, seed=1001, weight_law="zipf", zipf_s=1.5,
                nthreads=nthreads)


def scale24_graph(nthreads=None) -> CSRGraph:
    """R-MAT scale 24, edge factor 16, same quadrant probabilities, weights
    Zipf(1.2) clipped to [1, 10^4]."""
    return rmat(24, 16, 0.57, 0.19, 0.19, wmax=10000, seed=1002, weight_law="zipf", zipf_s=1.2,
                nthreads=nthreads)


def batch_specs(count: int = 64, meta_seed: int = 3000):
    """Parameters of the batch workload: per graph n log-uniform in
    [1e3, 1e6], mean degree uniform in [8, 24], exponent uniform in
    [2.1, 2.5], alpha in {0.1, 0.15, 0.2}, R in {64, 256}."""
    rng = np.random.Generator(np.random.Philox(meta_seed))
    specs = []
    for g in range(count):
        n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(1e6)))))
        deg = float(rng.uniform(8.0, 24.0))
        gamma = float(rng.uniform(2.1, 2.5))
        alpha = float(rng.choice([0.1, 0.15, 0.2]))
        R = int(rng.choice([64, 256]))
        specs.append(dict(index=g, n=n, m=int(round(n * deg)), gamma=gamma, alpha=alpha, R=R,
                          gen_seed=2000 + g, walk_seed=4000 + g, wmax=255))
    return specs


def batch_graph(spec, nthreads=None) -> CSRGraph:
    return chung_lu(spec["n"], spec["m"], spec["gamma"], spec["wmax"], seed=spec["gen_seed"],
                    weight_law="uniform", nthreads=nthreads)


def stratified_sources(g: CSRGraph, count: int, seed: int, hub_threshold: int = 4096,
                       small_max: int = 32) -> np.ndarray:
    """A source sample covering every node class: all hubs (capped at a
    quarter of the sample), a third small nodes, a third dangling nodes, the
    rest uniform. Sorted, unique, uint32."""
    deg = g.degrees()
    rng = np.random.Generator(np.random.Philox(seed))
    hubs = np.flatnonzero(deg > hub_threshold)
    if hubs.size > count // 4:
        hubs = rng.choice(hubs, count // 4, replace=False)
    small = np.flatnonzero((deg >= 1) & (deg <= small_max))
    dang = np.flatnonzero(deg == 0)
    pick = [hubs]
    for pool in (small, dang):
        k = min(pool.size, count // 3)
        if k:
            pick.append(rng.choice(pool, k, replace=False))
    have = np.unique(np.concatenate(pick)) if pick else np.zeros(0, np.int64)
    rest = count - have.size
    if rest > 0:
        extra = rng.choice(g.n, min(g.n, rest * 2), replace=False)
        extra = np.setdiff1d(extra, have)[:rest]
        have = np.unique(np.concatenate([have, extra]))
    return have.astype(np.uint32)


def poisson_queries(n_nodes: int, count: int, qps: float, seed: int = 5000,
                    max_sources: int = 1024, r_lo: float = 1e3, r_hi: float = 1e5):
    """Serving stream: Poisson arrivals at `qps`; per query 1..max_sources
    sources uniform over the nodes and a walk budget log-uniform in
    [r_lo, r_hi]."""
    rng = np.random.Generator(np.random.Philox(seed))
    t = 0.0
    out = []
    for q in range(count):
        t += float(rng.exponential(1.0 / qps))
        ns = int(rng.integers(1, max_sources + 1))
        src = rng.integers(0, n_nodes, ns).astype(np.uint32)
        R = int(round(math.exp(rng.uniform(math.log(r_lo), math.log(r_hi)))))
        out.append(dict(id=q, arrival=t, sources=src, R=R, seed=q))
    return out
