"""Thin Python binding of the fppr C-ABI (include/fppr.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels. PyTorch provides device memory and streams. The functions keep
the C names; `Graph` and `run` are small conveniences over them.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfppr.so")

FPPR_OK = 0
FPPR_INVALID_ARGUMENT = 1
FPPR_OUT_OF_MEMORY = 2
FPPR_DEVICE_ERROR = 3
FPPR_NOT_READY = 4
FPPR_CAPACITY = 5
FPPR_CANCELLED = 6
FPPR_INTERNAL = 7
FPPR_MEM_HOST = 0
FPPR_MEM_DEVICE = 1
FPPR_STITCH = 1
FPPR_COUNTS = 2
FPPR_DIGESTS = 4
FPPR_STATS = 8
FPPR_BATCH_REBUILD = 1
FPPR_SERVE_CONTINUOUS = 0
FPPR_SERVE_FIFO = 1
FPPR_MOVE_CAP = 65536
FPPR_NO_NODE = 0xFFFFFFFF

STATS_FIELDS = ("walks", "moves", "steps", "capped", "dangling_moves", "plain_moves",
                "stitched_moves", "probe_log_sum")


class FpprError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fppr status {status}: {msg}")
        self.status = status


class fppr_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("m", ctypes.c_uint64), ("row_offsets", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("w", ctypes.c_void_p), ("mem", ctypes.c_int)]


FPPR_LAYOUT_AUTO = 0
FPPR_LAYOUT_WIDE = 1
FPPR_LAYOUT_NARROW = 2
FPPR_LAYOUT_GUIDE = 3


class fppr_graph_opts(ctypes.Structure):
    _fields_ = [("hub_threshold", ctypes.c_uint32), ("layout", ctypes.c_uint32)]


class fppr_pool_opts(ctypes.Structure):
    _fields_ = [("S", ctypes.c_uint32), ("L", ctypes.c_uint32), ("K", ctypes.c_uint32),
                ("alpha", ctypes.c_double), ("seed", ctypes.c_uint64)]


class fppr_params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("R", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("topk", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("blocks_per_cu", ctypes.c_uint32)]


class fppr_out(ctypes.Structure):
    _fields_ = [("topk", ctypes.c_void_p), ("counts", ctypes.c_void_p),
                ("n_distinct", ctypes.c_void_p), ("digest", ctypes.c_void_p),
                ("endpoints", ctypes.c_void_p), ("stats", ctypes.c_void_p),
                ("profile", ctypes.c_void_p)]


class fppr_batch_item(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_void_p), ("params", fppr_params), ("sources", ctypes.c_void_p),
                ("n_sources", ctypes.c_uint64), ("out", fppr_out)]


class fppr_batch_opts(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32)]


class fppr_tune_space(ctypes.Structure):
    _fields_ = [("hub_thresholds", ctypes.c_void_p), ("n_hub_thresholds", ctypes.c_uint32),
                ("blocks_per_cu", ctypes.c_void_p), ("n_blocks_per_cu", ctypes.c_uint32),
                ("pools", ctypes.c_void_p), ("n_pools", ctypes.c_uint32),
                ("allow_plain", ctypes.c_uint32), ("n_sources", ctypes.c_uint64),
                ("sample", ctypes.c_uint32), ("reps", ctypes.c_uint32)]


class fppr_tune_result(ctypes.Structure):
    _fields_ = [("hub_threshold", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32),
                ("pool", ctypes.c_int32), ("trials", ctypes.c_uint32),
                ("est_ms", ctypes.c_double), ("plain_est_ms", ctypes.c_double)]


class fppr_server_opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_uint32), ("max_requests", ctypes.c_uint32),
                ("memory_bytes", ctypes.c_uint64), ("host_bytes", ctypes.c_uint64),
                ("slice_walks", ctypes.c_uint64), ("blocks_per_cu", ctypes.c_uint32)]


class fppr_query(ctypes.Structure):
    _fields_ = [("sources", ctypes.c_void_p), ("n_sources", ctypes.c_uint32), ("R", ctypes.c_uint32),
                ("alpha", ctypes.c_double), ("seed", ctypes.c_uint64), ("topk", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


class fppr_query_info(ctypes.Structure):
    _fields_ = [("submit_ns", ctypes.c_uint64), ("admit_ns", ctypes.c_uint64),
                ("done_ns", ctypes.c_uint64), ("walks", ctypes.c_uint64)]


class fppr_stats_t(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in ("walks", "moves", "steps", "capped", "dangling_moves",
                                               "plain_moves", "stitched_moves", "probe_log_sum")]


class fppr_server_counters(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("slices", ctypes.c_uint64), ("walk_launches", ctypes.c_uint64),
                ("peak_in_flight", ctypes.c_uint64), ("peak_device_bytes", ctypes.c_uint64),
                ("walk_stats", fppr_stats_t), ("cancelled", ctypes.c_uint64)]


class fppr_latency(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("max_ms", ctypes.c_double), ("span_s", ctypes.c_double),
                ("qps", ctypes.c_double)]


_lib = None

# (name, restype, argtypes) of every exported symbol
P = ctypes.c_void_p
_SIGS = [
    ("fppr_graph_create", ctypes.c_int, [ctypes.POINTER(fppr_csr), ctypes.POINTER(fppr_graph_opts), P,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    ("fppr_graph_destroy", ctypes.c_int, [P]),
    ("fppr_graph_rebuild", ctypes.c_int, [P, P]),
    ("fppr_graph_set_hub_threshold", ctypes.c_int, [P, ctypes.c_uint32, P]),
    ("fppr_graph_check", ctypes.c_int, [P, P]),
    ("fppr_graph_info", ctypes.c_int, [P, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64),
                                       ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64),
                                       ctypes.POINTER(ctypes.c_uint64)]),
    ("fppr_graph_layout", ctypes.c_int, [P, ctypes.POINTER(ctypes.c_uint32)]),
    ("fppr_graph_build_pool", ctypes.c_int, [P, ctypes.POINTER(fppr_pool_opts), P]),
    ("fppr_graph_export_pool", ctypes.c_int, [P, P, ctypes.c_uint64, P]),
    ("fppr_graph_alias_tables", ctypes.c_int, [P, P, P, P, P]),
    ("fppr_run_big_moves", ctypes.c_int, [P, P, P, P, P, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_double, ctypes.c_uint32, ctypes.c_uint64, P,
                                          ctypes.c_uint64, P, P, P]),
    ("fppr_graph_big_moves", ctypes.c_int, [P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                            ctypes.c_double, P, P, P, P, ctypes.c_uint64, P]),
    ("fppr_graph_alias_slots", ctypes.c_int, [P, P, P, P, P]),
    ("fppr_graph_alias_nodes", ctypes.c_int, [P, P, P]),
    ("fppr_run_alias", ctypes.c_int, [P, P, P, ctypes.c_double, ctypes.c_uint32, ctypes.c_uint64, P,
                                      ctypes.c_uint64, P, P, P]),
    ("fppr_alpha_threshold", ctypes.c_uint32, [ctypes.c_double]),
    ("fppr_walks_for_guarantee", ctypes.c_uint64, [ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    ("fppr_plan", ctypes.c_int, [P, ctypes.POINTER(fppr_params), ctypes.c_uint64,
                                 ctypes.POINTER(ctypes.c_uint64)]),
    ("fppr_plan_block", ctypes.c_int, [P, ctypes.POINTER(fppr_params), ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]),
    ("fppr_run", ctypes.c_int, [P, ctypes.POINTER(fppr_params), P, ctypes.c_uint64, P, ctypes.c_uint64,
                                ctypes.POINTER(fppr_out), P]),
    ("fppr_run_check", ctypes.c_int, [P, P]),
    ("fppr_aggregate_plan", ctypes.c_int, [ctypes.POINTER(fppr_params), ctypes.c_uint64,
                                           ctypes.POINTER(ctypes.c_uint64)]),
    ("fppr_aggregate", ctypes.c_int, [ctypes.POINTER(fppr_params), P, P, ctypes.c_uint64, P, ctypes.c_uint64,
                                      ctypes.POINTER(fppr_out), P]),
    ("fppr_run_static", ctypes.c_int, [P, ctypes.POINTER(fppr_params), P, ctypes.c_uint64,
                                       ctypes.POINTER(fppr_out), P]),
    ("fppr_profile_create", ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p)]),
    ("fppr_profile_destroy", ctypes.c_int, [P]),
    ("fppr_profile_read", ctypes.c_int, [P, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]),
    ("fppr_profile_read_walk", ctypes.c_int, [P, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_double)]),
    ("fppr_batch_plan", ctypes.c_int, [P, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint64)]),
    ("fppr_batch_create", ctypes.c_int, [P, ctypes.c_uint32, ctypes.POINTER(fppr_batch_opts), P,
                                         ctypes.c_uint64, ctypes.POINTER(ctypes.c_void_p)]),
    ("fppr_batch_run", ctypes.c_int, [P, P, P, P]),
    ("fppr_batch_capture", ctypes.c_int, [P, P, P]),
    ("fppr_batch_launch", ctypes.c_int, [P, P]),
    ("fppr_batch_check", ctypes.c_int, [P, P]),
    ("fppr_batch_destroy", ctypes.c_int, [P]),
    ("fppr_autotune", ctypes.c_int, [P, ctypes.POINTER(fppr_params), ctypes.POINTER(fppr_tune_space),
                                     ctypes.POINTER(fppr_tune_result), P]),
    ("fppr_server_create", ctypes.c_int, [P, ctypes.POINTER(fppr_server_opts), ctypes.POINTER(ctypes.c_void_p)]),
    ("fppr_server_submit", ctypes.c_int, [P, ctypes.POINTER(fppr_query), ctypes.POINTER(ctypes.c_uint64)]),
    ("fppr_server_poll", ctypes.c_int, [P, ctypes.c_uint64, P, P, ctypes.POINTER(fppr_query_info)]),
    ("fppr_server_wait", ctypes.c_int, [P, ctypes.c_uint64, P, P, ctypes.POINTER(fppr_query_info)]),
    ("fppr_server_stats", ctypes.c_int, [P, ctypes.POINTER(fppr_server_counters)]),
    ("fppr_server_destroy", ctypes.c_int, [P]),
    ("fppr_server_cancel", ctypes.c_int, [P, ctypes.c_uint64]),
    ("fppr_server_latency", ctypes.c_int, [P, ctypes.c_uint64, ctypes.POINTER(fppr_latency)]),
    ("fppr_batch_manifest", ctypes.c_int, [P, ctypes.c_char_p, ctypes.c_size_t,
                                           ctypes.POINTER(ctypes.c_size_t)]),
    ("fppr_last_error", ctypes.c_char_p, []),
]


def lib():
    """Loads the in-tree libfppr.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FpprError(FPPR_INTERNAL, f"{LIB_PATH} is missing: build it first "
                            "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return [name for name, _, _ in _SIGS]


def _check(status):
    if status != FPPR_OK:
        raise FpprError(status, lib().fppr_last_error().decode())


def fppr_alpha_threshold(alpha: float) -> int:
    return int(lib().fppr_alpha_threshold(float(alpha)))


def fppr_walks_for_guarantee(eps: float, delta: float, pf: float) -> int:
    return int(lib().fppr_walks_for_guarantee(eps, delta, pf))


def _stream_ptr(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def run_alias(graph, nodes, slots, alpha: float, R: int, seed: int, sources=None, steps=True, stream=None):
    """Walks that pick with alias tables (fppr_run_alias). nodes, slots: the
    tensors Graph.alias_nodes and Graph.alias_slots returned. sources: None (every node), a numpy
    uint32 array or a device int32 tensor. Returns device int32 tensors
    (endpoints, steps or None) of n_sources * R walks, walk-major per source."""
    import torch

    n = graph.info()["n"]
    if sources is None:
        src, n_src = None, n
    else:
        src = sources if isinstance(sources, torch.Tensor) else torch.from_numpy(
            np.ascontiguousarray(sources, dtype=np.uint32).view(np.int32)).cuda()
        n_src = int(src.numel())
    ep = torch.empty(max(n_src * R, 1), dtype=torch.int32, device="cuda")
    st = torch.empty(max(n_src * R, 1), dtype=torch.int32, device="cuda") if steps else None
    _check(lib().fppr_run_alias(graph.handle, _dptr(nodes), _dptr(slots), float(alpha), int(R), int(seed),
                                _dptr(src), n_src, _dptr(ep), _dptr(st), _stream_ptr(stream)))
    return ep[:n_src * R], (st[:n_src * R] if st is not None else None)


def run_big_moves(graph, slots, bm, S: int, alpha: float, R: int, seed: int, sources=None,
                  steps=True, stream=None):
    """Walks of the paper's design (fppr_run_big_moves). slots: from
    Graph.alias_slots; bm: the (entries, weights, counts) Graph.big_moves
    returned for the same S. Returns device int32 tensors (endpoints, steps
    or None) of n_sources * R walks, walk-major per source."""
    import torch

    ent, wts, cnt = bm
    n = graph.info()["n"]
    if sources is None:
        src, n_src = None, n
    else:
        src = sources if isinstance(sources, torch.Tensor) else torch.from_numpy(
            np.ascontiguousarray(sources, dtype=np.uint32).view(np.int32)).cuda()
        n_src = int(src.numel())
    ep = torch.empty(max(n_src * R, 1), dtype=torch.int32, device="cuda")
    st = torch.empty(max(n_src * R, 1), dtype=torch.int32, device="cuda") if steps else None
    _check(lib().fppr_run_big_moves(graph.handle, _dptr(slots), _dptr(ent), _dptr(wts), _dptr(cnt),
                                    int(ent.shape[1]), int(S), float(alpha), int(R), int(seed), _dptr(src),
                                    n_src, _dptr(ep), _dptr(st), _stream_ptr(stream)))
    return ep[:n_src * R], (st[:n_src * R] if st is not None else None)


class Graph:
    """Device graph. `csr` is a CSR object with n, row_offsets, col, w (numpy
    arrays: copied) or torch device tensors (borrowed: kept referenced here)."""

    def __init__(self, csr=None, hub_threshold: int = 0, stream=None, *, n=None,
                 row_offsets=None, col=None, w=None, layout: int = FPPR_LAYOUT_AUTO):
        import torch

        if csr is not None:
            n, row_offsets, col, w = csr.n, csr.row_offsets, csr.col, csr.w
        self.n = int(n)
        self._keep = None
        c = fppr_csr()
        c.n = self.n
        c.m = int(col.shape[0])
        if isinstance(col, torch.Tensor):
            assert row_offsets.dtype == torch.int64 and col.dtype == torch.int32 and w.dtype == torch.int32
            assert row_offsets.is_cuda and col.is_cuda and w.is_cuda
            self._keep = (row_offsets, col, w)
            c.row_offsets, c.col, c.w = _dptr(row_offsets), _dptr(col), _dptr(w)
            c.mem = FPPR_MEM_DEVICE
        else:
            ro = np.ascontiguousarray(row_offsets, dtype=np.uint64)
            cl = np.ascontiguousarray(col, dtype=np.uint32)
            ww = np.ascontiguousarray(w, dtype=np.uint32)
            self._host = (ro, cl, ww)
            c.row_offsets = ro.ctypes.data
            c.col = cl.ctypes.data if cl.size else None
            c.w = ww.ctypes.data if ww.size else None
            c.mem = FPPR_MEM_HOST
        self.m = int(c.m)
        o = fppr_graph_opts(hub_threshold, layout)
        h = ctypes.c_void_p()
        _check(lib().fppr_graph_create(ctypes.byref(c), ctypes.byref(o), _stream_ptr(stream),
                                       ctypes.byref(h)))
        self._h = h
        self._host = None
        self.pool_opts = None

    @property
    def handle(self):
        return self._h

    def info(self):
        n = ctypes.c_uint32()
        m = ctypes.c_uint64()
        hubs = ctypes.c_uint32()
        small = ctypes.c_uint64()
        by = ctypes.c_uint64()
        _check(lib().fppr_graph_info(self._h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(hubs),
                                     ctypes.byref(small), ctypes.byref(by)))
        return dict(n=n.value, m=m.value, hubs=hubs.value, small=small.value, device_bytes=by.value)

    def layout(self) -> int:
        """FPPR_LAYOUT_WIDE, FPPR_LAYOUT_NARROW or FPPR_LAYOUT_GUIDE."""
        v = ctypes.c_uint32()
        _check(lib().fppr_graph_layout(self._h, ctypes.byref(v)))
        return int(v.value)

    def build_pool(self, S: int, L: int, K: int, alpha: float, seed: int, stream=None):
        o = fppr_pool_opts(S, L, K, alpha, seed)
        _check(lib().fppr_graph_build_pool(self._h, ctypes.byref(o), _stream_ptr(stream)))
        self.pool_opts = dict(S=S, L=L, K=K, alpha=alpha, seed=seed)

    def export_pool(self, stream=None) -> np.ndarray:
        info = self.info()
        count = info["small"] * self.pool_opts["K"]
        out = np.zeros(max(count, 1), dtype=np.uint64)
        _check(lib().fppr_graph_export_pool(self._h, out.ctypes.data, count, _stream_ptr(stream)))
        return out[:count]

    def alias_tables(self, stream=None):
        """Alias tables of every row (fppr_graph_alias_tables): device tensors
        P (int64 holding the u64 thresholds) and alias (int32 holding u32
        in-row indices), indexed like the CSR's edges."""
        import torch

        m = self.info()["m"]
        P = torch.empty(max(m, 1), dtype=torch.int64, device="cuda")
        al = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
        scratch = torch.empty(max(2 * m, 1), dtype=torch.int32, device="cuda")
        _check(lib().fppr_graph_alias_tables(self._h, _dptr(P), _dptr(al), _dptr(scratch),
                                             _stream_ptr(stream)))
        self._alias_scratch = scratch  # kept alive until the next call; the launch is asynchronous
        return P[:m], al[:m]

    def alias_slots(self, P, alias, stream=None):
        """Packed 16-byte alias slots (fppr_graph_alias_slots) from the
        tensors alias_tables returned: a device int64 tensor [m, 2]."""
        import torch

        m = self.info()["m"]
        slots = torch.empty((max(m, 1), 2), dtype=torch.int64, device="cuda")
        _check(lib().fppr_graph_alias_slots(self._h, _dptr(P), _dptr(alias), _dptr(slots),
                                            _stream_ptr(stream)))
        return slots[:m]

    def alias_nodes(self, stream=None):
        """16-byte node records for the alias walks (fppr_graph_alias_nodes):
        a device int64 tensor [n, 2]."""
        import torch

        n = self.info()["n"]
        nodes = torch.empty((n, 2), dtype=torch.int64, device="cuda")
        _check(lib().fppr_graph_alias_nodes(self._h, _dptr(nodes), _stream_ptr(stream)))
        return nodes

    def big_moves(self, S: int, d: int, cap: int, alpha: float, slots: int = 16384, stream=None):
        """Exact big-move tables (fppr_graph_big_moves): device tensors
        entries and inclusive weight prefixes [n, cap] (int64 holding u64)
        and counts [n] (int32); node v's table is entries[v, :counts[v]]."""
        import torch

        n = self.info()["n"]
        ent = torch.zeros((n, cap), dtype=torch.int64, device="cuda")
        wts = torch.zeros((n, cap), dtype=torch.int64, device="cuda")
        cnt = torch.empty(n, dtype=torch.int32, device="cuda")
        scratch = torch.empty(8 * cap * max(1, min(slots, n)), dtype=torch.int64, device="cuda")
        _check(lib().fppr_graph_big_moves(self._h, int(S), int(d), int(cap), float(alpha), _dptr(ent),
                                          _dptr(wts), _dptr(cnt), _dptr(scratch), scratch.numel(),
                                          _stream_ptr(stream)))
        self._bm_scratch = scratch  # kept alive until the next call; the launch is asynchronous
        return ent, wts, cnt

    def rebuild(self, stream=None):
        _check(lib().fppr_graph_rebuild(self._h, _stream_ptr(stream)))

    def set_hub_threshold(self, hub_threshold: int, stream=None):
        _check(lib().fppr_graph_set_hub_threshold(self._h, int(hub_threshold), _stream_ptr(stream)))

    def autotune(self, alpha, R, seed, hub_thresholds=None, blocks_per_cu=None, pools=(),
                 allow_plain=True, n_sources=0, sample=0, reps=0, stream=None):
        """Runs the library's autotuner (fppr_autotune). pools: sequence of
        dicts with S, L, K, seed. Returns the chosen configuration as a dict;
        the graph is left in it (pool built, or none)."""
        hs = np.asarray(hub_thresholds if hub_thresholds is not None else [], dtype=np.uint32)
        bs = np.asarray(blocks_per_cu if blocks_per_cu is not None else [], dtype=np.uint32)
        parr = (fppr_pool_opts * max(1, len(pools)))()
        for k, o in enumerate(pools):
            parr[k] = fppr_pool_opts(o["S"], o["L"], o["K"], float(alpha), o["seed"])
        sp = fppr_tune_space(hs.ctypes.data if hs.size else None, hs.size,
                             bs.ctypes.data if bs.size else None, bs.size,
                             ctypes.cast(parr, ctypes.c_void_p) if len(pools) else None, len(pools),
                             1 if allow_plain else 0, int(n_sources), int(sample), int(reps))
        p = make_params(alpha, R, seed, 0, False, False, False, False)
        r = fppr_tune_result()
        _check(lib().fppr_autotune(self._h, ctypes.byref(p), ctypes.byref(sp), ctypes.byref(r),
                                   _stream_ptr(stream)))
        chosen = dict(pools[r.pool]) if r.pool >= 0 else None
        if chosen is not None:
            self.pool_opts = dict(chosen, alpha=float(alpha))
        else:
            self.pool_opts = None
        return dict(hub_threshold=r.hub_threshold, blocks_per_cu=r.blocks_per_cu, pool=r.pool,
                    pool_opts=chosen, trials=r.trials, est_ms=r.est_ms, plain_est_ms=r.plain_est_ms)

    def check(self, stream=None):
        _check(lib().fppr_graph_check(self._h, _stream_ptr(stream)))

    def close(self):
        if getattr(self, "_h", None):
            lib().fppr_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_params(alpha, R, seed, topk=0, stitch=False, counts=True, digests=True, stats=True,
                blocks_per_cu=0):
    flags = (FPPR_STITCH if stitch else 0) | (FPPR_COUNTS if counts else 0) | \
        (FPPR_DIGESTS if digests else 0) | (FPPR_STATS if stats else 0)
    return fppr_params(float(alpha), int(R), int(seed), int(topk), flags, int(blocks_per_cu))


def fppr_plan_block(graph: Graph, params: fppr_params, n_sources: int, budget: int):
    """(block_sources, workspace_bytes) of a memory-bounded run."""
    b = ctypes.c_uint64()
    ws = ctypes.c_uint64()
    _check(lib().fppr_plan_block(graph.handle, ctypes.byref(params), n_sources, budget, ctypes.byref(b),
                                 ctypes.byref(ws)))
    return int(b.value), int(ws.value)


def fppr_plan(graph: Graph, params: fppr_params, n_sources: int) -> int:
    ws = ctypes.c_uint64()
    _check(lib().fppr_plan(graph.handle, ctypes.byref(params), n_sources, ctypes.byref(ws)))
    return int(ws.value)


@dataclass
class Outputs:
    topk: object = None        # torch int32 [n_src, k, 2] (bit pattern of uint32)
    counts: object = None      # torch int32 [n_src, R, 2]
    n_distinct: object = None  # torch int32 [n_src]
    digest: object = None      # torch int64 [n_src]
    endpoints: object = None   # torch int32 [n_src, R]
    stats: object = None       # torch int64 [8]
    profile: object = None     # Profile (stage timer) or None

    def stats_dict(self):
        if self.stats is None:
            return None
        v = self.stats.cpu().numpy().astype(np.uint64)
        return {k: int(x) for k, x in zip(STATS_FIELDS, v)}


def alloc_outputs(n_src, R, topk, counts=True, digests=True, stats=True, endpoints=False,
                  device="cuda"):
    import torch

    o = Outputs()
    if topk:
        o.topk = torch.empty((n_src, topk, 2), dtype=torch.int32, device=device)
    if counts:
        o.counts = torch.empty((n_src, R, 2), dtype=torch.int32, device=device)
        o.n_distinct = torch.empty((n_src,), dtype=torch.int32, device=device)
    if digests:
        o.digest = torch.empty((n_src,), dtype=torch.int64, device=device)
    if stats:
        o.stats = torch.zeros((8,), dtype=torch.int64, device=device)
    if endpoints:
        o.endpoints = torch.empty((n_src, R), dtype=torch.int32, device=device)
    return o


def fppr_run(graph: Graph, params: fppr_params, sources, n_sources: int, workspace, out: Outputs,
             stream=None):
    """sources: torch int32 device tensor or None (all nodes)."""
    o = fppr_out(_dptr(out.topk), _dptr(out.counts), _dptr(out.n_distinct), _dptr(out.digest),
                 _dptr(out.endpoints), _dptr(out.stats),
                 out.profile.handle if out.profile is not None else None)
    _check(lib().fppr_run(graph.handle, ctypes.byref(params), _dptr(sources), n_sources,
                          _dptr(workspace), workspace.numel() * workspace.element_size(),
                          ctypes.byref(o), _stream_ptr(stream)))


def fppr_run_static(graph: Graph, params: fppr_params, sources, n_sources: int, out: Outputs,
                    stream=None):
    """fppr_run with the library's fixed device workspace (no allocation in
    the library). sources: torch int32 device tensor or None (all nodes)."""
    o = fppr_out(_dptr(out.topk), _dptr(out.counts), _dptr(out.n_distinct), _dptr(out.digest),
                 _dptr(out.endpoints), _dptr(out.stats),
                 out.profile.handle if out.profile is not None else None)
    _check(lib().fppr_run_static(graph.handle, ctypes.byref(params), _dptr(sources), n_sources,
                                 ctypes.byref(o), _stream_ptr(stream)))


def count(endpoints, R, topk, sources=None, n_sources=None, counts=True, digests=True, stream=None) -> Outputs:
    """fppr_aggregate over device endpoints (int32 tensor, n_sources * R):
    counting, top-k and digests as fppr_run computes them. sources: None
    (row j is node j) or a device int32 tensor / int sequence of source ids."""
    import torch

    src = None
    if sources is not None:
        src = sources if isinstance(sources, torch.Tensor) else torch.from_numpy(
            np.ascontiguousarray(sources, dtype=np.uint32).view(np.int32)).cuda()
        n_sources = int(src.numel())
    n_sources = int(n_sources if n_sources is not None else endpoints.numel() // R)
    p = make_params(0.5, R, 0, topk, False, counts, digests, False)
    ws_bytes = ctypes.c_uint64()
    _check(lib().fppr_aggregate_plan(ctypes.byref(p), n_sources, ctypes.byref(ws_bytes)))
    ws = torch.empty((ws_bytes.value + 7) // 8, dtype=torch.int64, device="cuda")
    out = alloc_outputs(n_sources, R, topk, counts, digests, stats=False)
    o = fppr_out(_dptr(out.topk), _dptr(out.counts), _dptr(out.n_distinct), _dptr(out.digest), None, None, None)
    _check(lib().fppr_aggregate(ctypes.byref(p), _dptr(endpoints), _dptr(src), n_sources, _dptr(ws),
                                ws.numel() * 8, ctypes.byref(o), _stream_ptr(stream)))
    out._workspace = ws
    return out


class Profile:
    """Stage timer: walk and aggregation kernel durations of the last run."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(lib().fppr_profile_create(ctypes.byref(h)))
        self.handle = h

    def read(self):
        a = ctypes.c_double()
        b = ctypes.c_double()
        _check(lib().fppr_profile_read(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def read_walk(self):
        """(walk kernel ms, coin-only kernel ms) of the last single-launch run."""
        a = ctypes.c_double()
        b = ctypes.c_double()
        _check(lib().fppr_profile_read_walk(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def __del__(self):
        if getattr(self, "handle", None):
            lib().fppr_profile_destroy(self.handle)
            self.handle = None


def fppr_run_check(workspace, stream=None):
    _check(lib().fppr_run_check(_dptr(workspace), _stream_ptr(stream)))


def run(graph: Graph, alpha, R, seed, sources=None, topk=0, stitch=False, counts=True,
        digests=True, stats=True, endpoints=False, stream=None, check=True, blocks_per_cu=0,
        max_workspace=None) -> Outputs:
    """Allocates workspace and outputs with torch, runs, and returns the outputs
    (device tensors). sources: None (all nodes) or an int sequence / tensor."""
    import torch

    if sources is None:
        src = None
        n_src = graph.n
    else:
        src = torch.as_tensor(np.asarray(sources, dtype=np.uint32).view(np.int32)
                              if not isinstance(sources, torch.Tensor) else sources)
        src = src.to(device="cuda", dtype=torch.int32).contiguous()
        n_src = int(src.numel())
    p = make_params(alpha, R, seed, topk, stitch, counts, digests, stats, blocks_per_cu)
    ws_bytes = fppr_plan(graph, p, n_src)
    if max_workspace is not None and max_workspace < ws_bytes:
        _, ws_bytes = fppr_plan_block(graph, p, n_src, max_workspace)
    ws = torch.empty((ws_bytes + 7) // 8, dtype=torch.int64, device="cuda")
    out = alloc_outputs(n_src, R, topk, counts, digests, stats, endpoints)
    fppr_run(graph, p, src, n_src, ws, out, stream)
    if check:
        fppr_run_check(ws, stream)
    out._workspace = ws
    return out


class Batch:
    """Several (graph, params, sources) items in one persistent walk launch.
    items: list of dicts with keys graph (Graph), alpha, R, seed, topk,
    stitch, sources (None or int sequence), counts, digests. Outputs are
    allocated here (torch) as Outputs objects in `self.outputs`."""

    def __init__(self, items, counts=True, digests=True, stats=True, rebuild=False, blocks_per_cu=0):
        import torch

        self._keep = []
        arr = (fppr_batch_item * len(items))()
        self.outputs = []
        for k, it in enumerate(items):
            G = it["graph"]
            if it.get("sources") is None:
                src, n_src = None, G.n
            else:
                src = torch.as_tensor(np.asarray(it["sources"], dtype=np.uint32).view(np.int32)).cuda()
                n_src = int(src.numel())
            p = make_params(it["alpha"], it["R"], it["seed"], it.get("topk", 0), it.get("stitch", False),
                            counts, digests, False)
            o = alloc_outputs(n_src, it["R"], it.get("topk", 0), counts, digests, False)
            self.outputs.append(o)
            self._keep.append((G, src))
            arr[k].graph = G.handle
            arr[k].params = p
            arr[k].sources = _dptr(src)
            arr[k].n_sources = n_src
            arr[k].out = fppr_out(_dptr(o.topk), _dptr(o.counts), _dptr(o.n_distinct), _dptr(o.digest),
                                  None, None, None)
        self._items = arr
        ws = ctypes.c_uint64()
        _check(lib().fppr_batch_plan(arr, len(items), ctypes.byref(ws)))
        self.workspace = torch.empty((ws.value + 7) // 8, dtype=torch.int64, device="cuda")
        self.stats = torch.zeros(8, dtype=torch.int64, device="cuda") if stats else None
        h = ctypes.c_void_p()
        opts = fppr_batch_opts(FPPR_BATCH_REBUILD if rebuild else 0, int(blocks_per_cu))
        _check(lib().fppr_batch_create(arr, len(items), ctypes.byref(opts), _dptr(self.workspace), ws.value,
                                       ctypes.byref(h)))
        self._h = h

    def stats_dict(self):
        if self.stats is None:
            return None
        v = self.stats.cpu().numpy().astype(np.uint64)
        return {k: int(x) for k, x in zip(STATS_FIELDS, v)}

    def run(self, stream=None, profile=None):
        _check(lib().fppr_batch_run(self._h, _dptr(self.stats),
                                    profile.handle if profile is not None else None,
                                    _stream_ptr(stream)))

    def capture(self, stream):
        _check(lib().fppr_batch_capture(self._h, _dptr(self.stats), _stream_ptr(stream)))

    def launch(self, stream=None):
        _check(lib().fppr_batch_launch(self._h, _stream_ptr(stream)))

    def check(self, stream=None):
        _check(lib().fppr_batch_check(self._h, _stream_ptr(stream)))

    def manifest(self) -> dict:
        """The library's run manifest (fppr_batch_manifest) as a dict."""
        import json

        need = ctypes.c_size_t()
        _check(lib().fppr_batch_manifest(self._h, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        _check(lib().fppr_batch_manifest(self._h, buf, need.value, ctypes.byref(need)))
        return json.loads(buf.value.decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().fppr_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """A resident-graph query server (fppr_server_*). mode: "continuous" or
    "fifo". submit() returns an id; poll()/wait() return (topk, digest, info)
    with topk uint32 [n_sources, k, 2] and digest uint64 [n_sources], or None
    from poll() while the query runs."""

    def __init__(self, graph: Graph, mode="continuous", max_requests=64, memory_bytes=16 << 30,
                 host_bytes=256 << 20, slice_walks=1 << 26, blocks_per_cu=0):
        o = fppr_server_opts(FPPR_SERVE_FIFO if mode == "fifo" else FPPR_SERVE_CONTINUOUS, max_requests,
                             memory_bytes, host_bytes, slice_walks, blocks_per_cu)
        h = ctypes.c_void_p()
        _check(lib().fppr_server_create(graph.handle, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._graph = graph
        self._shape = {}

    def submit(self, sources, R, alpha, seed, topk, stitch=False) -> int:
        src = np.ascontiguousarray(sources, dtype=np.uint32)
        q = fppr_query(src.ctypes.data, src.size, int(R), float(alpha), int(seed), int(topk),
                       FPPR_STITCH if stitch else 0)
        qid = ctypes.c_uint64()
        _check(lib().fppr_server_submit(self._h, ctypes.byref(q), ctypes.byref(qid)))
        self._shape[qid.value] = (src.size, int(topk))
        return qid.value

    def _take(self, fn, qid):
        if qid not in self._shape:
            raise FpprError(FPPR_INVALID_ARGUMENT, "unknown query id")
        n, k = self._shape[qid]
        topk = np.empty((n, k, 2), dtype=np.uint32)
        digest = np.empty(n, dtype=np.uint64)
        info = fppr_query_info()
        st = fn(self._h, qid, topk.ctypes.data, digest.ctypes.data, ctypes.byref(info))
        if st == FPPR_NOT_READY:
            return None
        if st == FPPR_CANCELLED:
            del self._shape[qid]
        _check(st)
        del self._shape[qid]
        return topk, digest, dict(submit_ns=info.submit_ns, admit_ns=info.admit_ns, done_ns=info.done_ns,
                                  walks=info.walks)

    def poll(self, qid):
        return self._take(lib().fppr_server_poll, qid)

    def wait(self, qid):
        return self._take(lib().fppr_server_wait, qid)

    def cancel(self, qid):
        """fppr_server_cancel: poll/wait of qid then raise FpprError(FPPR_CANCELLED)."""
        _check(lib().fppr_server_cancel(self._h, int(qid)))

    def latency(self, first_id=0):
        """fppr_server_latency over completed queries with id >= first_id."""
        lt = fppr_latency()
        _check(lib().fppr_server_latency(self._h, int(first_id), ctypes.byref(lt)))
        return {f: getattr(lt, f) for f, _ in fppr_latency._fields_}

    def stats(self):
        st = fppr_server_counters()
        _check(lib().fppr_server_stats(self._h, ctypes.byref(st)))
        d = {f: getattr(st, f) for f, _ in fppr_server_counters._fields_ if f != "walk_stats"}
        d["walk_stats"] = {f: getattr(st.walk_stats, f) for f, _ in fppr_stats_t._fields_}
        return d

    def close(self):
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            _check(lib().fppr_server_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
