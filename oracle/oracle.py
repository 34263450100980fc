"""ctypes wrapper of the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module. It loads `liboracle.so`, built from `fppr_oracle.c` with gcc;
it never touches the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "fppr_oracle.c")
_lib = None

MOVE_CAP = 65536
POOL_TERM = 1


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", "-pthread",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in (
        "walks", "moves", "steps", "capped", "dangling_moves", "plain_moves", "stitched_moves",
        "probe_log_sum", "lines")]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    lib.or_philox4x32_10.argtypes = [P, P, P]
    lib.or_alpha_threshold.argtypes = [ctypes.c_double]
    lib.or_alpha_threshold.restype = u32
    lib.or_pick.argtypes = [P, u32, u32, u32]
    lib.or_pick.restype = u32
    lib.or_graph_new.argtypes = [u32, u64, P, P, P]
    lib.or_graph_new.restype = P
    lib.or_graph_free.argtypes = [P]
    lib.or_graph_prefix.argtypes = [P, P]
    lib.or_pool_new.argtypes = [P, u32, u32, u32, u32, u64, i32]
    lib.or_pool_new.restype = P
    lib.or_pool_free.argtypes = [P]
    lib.or_pool_small_count.argtypes = [P]
    lib.or_pool_small_count.restype = u64
    lib.or_pool_entries.argtypes = [P, P]
    lib.or_run.argtypes = [P, P, u32, u64, u32, P, u64, u32, i32, P, P, P, P, P, P,
                           ctypes.POINTER(Stats)]
    lib.or_run.restype = i32
    lib.or_digest_term.argtypes = [u32, u32, u32]
    lib.or_digest_term.restype = u64
    _lib = lib
    return lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().or_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def alpha_threshold(alpha: float) -> int:
    return int(_load().or_alpha_threshold(float(alpha)))


def pick(prefix_row, x0: int, x1: int) -> int:
    P = np.ascontiguousarray(prefix_row, dtype=np.uint64)
    return int(_load().or_pick(_p(P), P.shape[0], x0, x1))


def digest_term(s: int, t: int, c: int) -> int:
    return int(_load().or_digest_term(s, t, c))


class Graph:
    """Oracle view of a CSR graph (keeps references to the caller's arrays)."""

    def __init__(self, n, row_offsets, col, w):
        self.n = int(n)
        self.row_offsets = np.ascontiguousarray(row_offsets, dtype=np.uint64)
        self.col = np.ascontiguousarray(col, dtype=np.uint32)
        self.w = np.ascontiguousarray(w, dtype=np.uint32)
        self.m = int(self.col.shape[0])
        self._h = _load().or_graph_new(self.n, self.m, _p(self.row_offsets), _p(self.col),
                                       _p(self.w))
        if not self._h:
            raise ValueError("invalid CSR graph")

    @classmethod
    def from_csr(cls, g):
        return cls(g.n, g.row_offsets, g.col, g.w)

    def prefix(self) -> np.ndarray:
        out = np.empty(max(self.m, 1), dtype=np.uint64)
        _load().or_graph_prefix(self._h, _p(out))
        return out[: self.m]

    def __del__(self):
        if getattr(self, "_h", None):
            _load().or_graph_free(self._h)
            self._h = None


class Pool:
    """Short-walk pool of the small nodes (1 <= deg <= S)."""

    def __init__(self, graph: Graph, S: int, L: int, K: int, alpha: float, seed: int,
                 nthreads: int | None = None):
        self.graph = graph
        self.S, self.L, self.K, self.seed = S, L, K, seed
        self.T = alpha_threshold(alpha)
        self._h = _load().or_pool_new(graph._h, S, L, K, self.T, seed,
                                      nthreads or default_threads())
        if not self._h:
            raise ValueError("invalid pool parameters")

    @property
    def small_count(self) -> int:
        return int(_load().or_pool_small_count(self._h))

    def entries(self) -> np.ndarray:
        out = np.empty(max(self.small_count * self.K, 1), dtype=np.uint64)
        _load().or_pool_entries(self._h, _p(out))
        return out[: self.small_count * self.K]

    def __del__(self):
        if getattr(self, "_h", None):
            _load().or_pool_free(self._h)
            self._h = None


@dataclass
class RunResult:
    n_distinct: np.ndarray | None
    counts: np.ndarray | None      # [n_src, R, 2]
    topk: np.ndarray | None        # [n_src, k, 2]
    digest: np.ndarray | None      # [n_src]
    endpoints: np.ndarray | None   # [n_src, R]
    lengths: np.ndarray | None     # [n_src, R]
    stats: dict


def run(graph: Graph, alpha: float, R: int, seed: int, sources=None, topk: int = 0,
        pool: Pool | None = None, nthreads: int | None = None, want_counts=True,
        want_endpoints=False, want_lengths=False) -> RunResult:
    T = alpha_threshold(alpha)
    src = None if sources is None else np.ascontiguousarray(sources, dtype=np.uint32)
    n_src = graph.n if src is None else int(src.shape[0])
    nd = np.zeros(n_src, dtype=np.uint32)
    counts = np.zeros((n_src, R, 2), dtype=np.uint32) if want_counts else None
    tk = np.zeros((n_src, topk, 2), dtype=np.uint32) if topk else None
    dg = np.zeros(n_src, dtype=np.uint64)
    ep = np.zeros((n_src, R), dtype=np.uint32) if want_endpoints else None
    ln = np.zeros((n_src, R), dtype=np.uint32) if want_lengths else None
    st = Stats()
    rc = _load().or_run(graph._h, pool._h if pool else None, T, seed, R, _p(src), n_src, topk,
                        nthreads or default_threads(), _p(nd), _p(counts), _p(tk), _p(dg), _p(ep),
                        _p(ln), ctypes.byref(st))
    if rc != 0:
        raise ValueError("oracle run rejected its arguments")
    return RunResult(nd, counts, tk, dg, ep, ln, st.as_dict())
