"""Python binding of libgvl.so: GVE-Leiden's hot path as hand-written HIP for MI355X.

The functions named ``gvl_*`` mirror the C ABI of ``include/gvl.h`` one to
one and only marshal arguments (device pointers come from torch tensors,
the stream from ``torch.cuda.current_stream()``).  ``leiden`` and
``modularity`` are conveniences that also allocate the output and the
workspace as torch tensors.  Every step of the algorithm runs in the HIP
kernels; there is no CPU or PyTorch fallback: if libgvl.so is missing the
import of the library fails with an error.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgvl.so")

GVL_MODE_FAST = 0
GVL_MODE_DET = 1
GVL_MAX_PASS_STATS = 64

STATUS = {0: "GVL_OK", -1: "GVL_E_INVALID_ARG", -2: "GVL_E_BAD_CSR", -3: "GVL_E_NOT_SYMMETRIC",
          -4: "GVL_E_NONINTEGER_WEIGHT",
          -5: "GVL_E_RESOLUTION", -6: "GVL_E_WORKSPACE", -8: "GVL_E_HIP", -9: "GVL_E_BUSY", -10: "GVL_E_BATCH",
          -11: "GVL_E_TABLE_OVERFLOW"}

GVL_REQ_PENDING, GVL_REQ_RUNNING, GVL_REQ_DONE, GVL_REQ_CANCELLED = 0, 1, 2, 3


class GvlError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__("%s returned %s (%d)" % (where, STATUS.get(code, "?"), code))
        self.code = code


class gvl_options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("tolerance", ctypes.c_double),
                ("tolerance_drop", ctypes.c_double), ("aggregation_tolerance", ctypes.c_double),
                ("max_iterations", ctypes.c_int32), ("max_passes", ctypes.c_int32),
                ("refine_sweeps", ctypes.c_int32), ("subsweeps", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("debug_trace", ctypes.c_int32), ("sync_moves", ctypes.c_int32),
                ("louvain", ctypes.c_int32), ("refine_random", ctypes.c_int32), ("seed", ctypes.c_uint32),
                ("shrink_excludes_isolated", ctypes.c_int32), ("no_graph_replay", ctypes.c_int32),
                ("refine_based", ctypes.c_int32)]


_P = GVL_MAX_PASS_STATS


class gvl_stats(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_int32), ("termination", ctypes.c_int32),
                ("num_communities", ctypes.c_int64),
                ("iterations", ctypes.c_int32 * _P), ("refine_sweeps", ctypes.c_int32 * _P),
                ("nv", ctypes.c_int64 * _P), ("ne", ctypes.c_int64 * _P), ("ncom", ctypes.c_int64 * _P),
                ("ms_move", ctypes.c_double), ("ms_refine", ctypes.c_double),
                ("ms_aggregate", ctypes.c_double), ("ms_other", ctypes.c_double),
                ("ms_total", ctypes.c_double),
                ("scan_vertices", ctypes.c_int64), ("scan_arcs", ctypes.c_int64),
                ("scan_candidates", ctypes.c_int64), ("scan_moves", ctypes.c_int64),
                ("agg_vertices", ctypes.c_int64), ("agg_arcs", ctypes.c_int64),
                ("agg_out_arcs", ctypes.c_int64),
                ("ms_scan_kernels", ctypes.c_double), ("ms_agg_kernels", ctypes.c_double),
                ("scan_launches", ctypes.c_int64), ("agg_launches", ctypes.c_int64),
                ("scan_refine_arcs", ctypes.c_int64), ("ms_scan_move_kernels", ctypes.c_double),
                ("graph_launches", ctypes.c_int64), ("table_overflows", ctypes.c_int64)]


class gvl_graph_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("d_offsets", ctypes.c_void_p),
                ("d_indices", ctypes.c_void_p), ("d_weights", ctypes.c_void_p), ("resolution", ctypes.c_double),
                ("d_membership", ctypes.c_void_p)]


class gvl_request_info(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("result", ctypes.c_int32), ("modularity", ctypes.c_double),
                ("latency_ms", ctypes.c_double), ("queue_ms", ctypes.c_double)]


class gvl_server_info(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("pending", ctypes.c_int64), ("running", ctypes.c_int64),
                ("max_running", ctypes.c_int64), ("arena_bytes", ctypes.c_size_t), ("arena_used", ctypes.c_size_t),
                ("arena_peak", ctypes.c_size_t)]


GVL_CLASS_SMALL, GVL_CLASS_LOWDEG, GVL_CLASS_SKEWED, GVL_CLASS_BATCH, GVL_NUM_CLASSES = 0, 1, 2, 3, 4
CLASS_NAMES = ("small", "lowdeg", "skewed", "batch")


class gvl_tuning(ctypes.Structure):
    _fields_ = [("bin_max", ctypes.c_int32 * 6), ("decide_grid", ctypes.c_int32), ("commit_grid", ctypes.c_int32),
                ("agg_grid", ctypes.c_int32)]


EXPORTS = ["gvl_create", "gvl_destroy", "gvl_default_options", "gvl_workspace_bytes", "gvl_leiden",
           "gvl_leiden_static", "gvl_graph_class", "gvl_get_tuning", "gvl_set_tuning", "gvl_load_tuning",
           "gvl_modularity", "gvl_disconnected_communities", "gvl_gather_probe", "gvl_debug_pass_info", "gvl_debug_export_pass", "gvl_debug_pass_movers",
           "gvl_batch_workspace_bytes", "gvl_leiden_batch", "gvl_fused_workspace_bytes", "gvl_leiden_fused",
           "gvl_server_create", "gvl_server_submit",
           "gvl_server_poll", "gvl_server_wait", "gvl_server_cancel", "gvl_server_release",
           "gvl_server_set_batching", "gvl_server_stats",
           "gvl_server_destroy", "gvl_status_string"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgvl.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError("libgvl.so not found at %s: build it with paper_2312_13936_amd/build.py" % path)
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    lib.gvl_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp]
    lib.gvl_destroy.argtypes = [vp]
    lib.gvl_default_options.argtypes = [ctypes.POINTER(gvl_options), i32]
    lib.gvl_workspace_bytes.argtypes = [i64, i64, ctypes.POINTER(gvl_options), ctypes.POINTER(sz)]
    lib.gvl_leiden.argtypes = [vp, i64, i64, vp, vp, vp, dbl, ctypes.POINTER(gvl_options), vp, sz, vp,
                               ctypes.POINTER(dbl), ctypes.POINTER(gvl_stats)]
    lib.gvl_leiden_static.argtypes = [vp, i64, i64, vp, vp, vp, dbl, ctypes.POINTER(gvl_options), vp,
                                      ctypes.POINTER(dbl), ctypes.POINTER(gvl_stats)]
    lib.gvl_graph_class.argtypes = [i64, i64, i32, ctypes.POINTER(i32)]
    lib.gvl_get_tuning.argtypes = [i32, ctypes.POINTER(gvl_tuning)]
    lib.gvl_set_tuning.argtypes = [i32, ctypes.POINTER(gvl_tuning)]
    lib.gvl_load_tuning.argtypes = [ctypes.c_char_p]
    lib.gvl_modularity.argtypes = [vp, i64, i64, vp, vp, vp, vp, dbl, vp, sz, ctypes.POINTER(dbl)]
    lib.gvl_gather_probe.argtypes = [vp, i64, i64, vp, i64, vp]
    lib.gvl_disconnected_communities.argtypes = [vp, i64, i64, vp, vp, vp, vp, sz, vp, ctypes.POINTER(i64)]
    lib.gvl_debug_pass_info.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.gvl_debug_export_pass.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    lib.gvl_debug_pass_movers.argtypes = [vp, i32, vp, i32, vp, i32]
    GD = ctypes.POINTER(gvl_graph_desc)
    lib.gvl_batch_workspace_bytes.argtypes = [i32, GD, ctypes.POINTER(gvl_options), i32, ctypes.POINTER(sz)]
    lib.gvl_leiden_batch.argtypes = [vp, i32, GD, ctypes.POINTER(gvl_options), i32, vp, sz,
                                     ctypes.POINTER(dbl), ctypes.POINTER(i32)]
    lib.gvl_fused_workspace_bytes.argtypes = [i32, GD, ctypes.POINTER(gvl_options), ctypes.POINTER(sz)]
    lib.gvl_leiden_fused.argtypes = [vp, i32, GD, ctypes.POINTER(gvl_options), vp, sz, ctypes.POINTER(dbl),
                                     ctypes.POINTER(i32)]
    lib.gvl_server_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, i32, ctypes.POINTER(gvl_options), vp, sz]
    lib.gvl_server_submit.argtypes = [vp, GD, ctypes.POINTER(ctypes.c_uint64)]
    lib.gvl_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(gvl_request_info)]
    lib.gvl_server_wait.argtypes = [vp, ctypes.c_uint64, i64, ctypes.POINTER(gvl_request_info)]
    lib.gvl_server_cancel.argtypes = [vp, ctypes.c_uint64]
    lib.gvl_server_release.argtypes = [vp, ctypes.c_uint64]
    lib.gvl_server_set_batching.argtypes = [vp, i32, i64]
    lib.gvl_server_stats.argtypes = [vp, ctypes.POINTER(gvl_server_info)]
    lib.gvl_server_destroy.argtypes = [vp]
    for f in EXPORTS[:-1]:
        getattr(lib, f).restype = ctypes.c_int
    lib.gvl_status_string.argtypes = [ctypes.c_int]
    lib.gvl_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(code: int, where: str):
    if code != 0:
        raise GvlError(code, where)


# ------------------------------------------------------------ C-ABI mirror ---

def gvl_create(device: int = 0, stream: Optional[int] = None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(load_library().gvl_create(ctypes.byref(h), device, stream), "gvl_create")
    return h


def gvl_destroy(ctx) -> None:
    _check(load_library().gvl_destroy(ctx), "gvl_destroy")


def gvl_default_options(mode: int = GVL_MODE_FAST) -> gvl_options:
    o = gvl_options()
    _check(load_library().gvl_default_options(ctypes.byref(o), mode), "gvl_default_options")
    return o


def gvl_workspace_bytes(n: int, m: int, opt: gvl_options) -> int:
    b = ctypes.c_size_t(0)
    _check(load_library().gvl_workspace_bytes(n, m, ctypes.byref(opt), ctypes.byref(b)), "gvl_workspace_bytes")
    return int(b.value)


def gvl_leiden(ctx, n, m, d_offsets, d_indices, d_weights, resolution, opt, d_workspace, workspace_bytes,
               d_membership, stats: Optional[gvl_stats] = None) -> float:
    q = ctypes.c_double(0.0)
    code = load_library().gvl_leiden(ctx, n, m, d_offsets, d_indices, d_weights, resolution, ctypes.byref(opt),
                                     d_workspace, workspace_bytes, d_membership, ctypes.byref(q),
                                     ctypes.byref(stats) if stats is not None else None)
    _check(code, "gvl_leiden")
    return q.value


def gvl_graph_class(n: int, m: int, fused: bool = False) -> int:
    c = ctypes.c_int32(0)
    _check(load_library().gvl_graph_class(n, m, 1 if fused else 0, ctypes.byref(c)), "gvl_graph_class")
    return c.value


def gvl_get_tuning(cls: int) -> gvl_tuning:
    t = gvl_tuning()
    _check(load_library().gvl_get_tuning(cls, ctypes.byref(t)), "gvl_get_tuning")
    return t


def gvl_set_tuning(cls: int, t: gvl_tuning) -> None:
    _check(load_library().gvl_set_tuning(cls, ctypes.byref(t)), "gvl_set_tuning")


def gvl_load_tuning(path: str) -> None:
    _check(load_library().gvl_load_tuning(path.encode()), "gvl_load_tuning")


GVL_STATIC_WORKSPACE_BYTES = 256 * 1024 * 1024


def gvl_leiden_static(ctx, n, m, d_offsets, d_indices, d_weights, resolution, opt, d_membership,
                      stats: Optional[gvl_stats] = None) -> float:
    """gvl_leiden with the library's own device array as workspace (no device
    allocation anywhere in the call); graphs whose workspace exceeds
    GVL_STATIC_WORKSPACE_BYTES are rejected with GVL_E_WORKSPACE."""
    q = ctypes.c_double(0.0)
    code = load_library().gvl_leiden_static(ctx, n, m, d_offsets, d_indices, d_weights, resolution,
                                            ctypes.byref(opt), d_membership, ctypes.byref(q),
                                            ctypes.byref(stats) if stats is not None else None)
    _check(code, "gvl_leiden_static")
    return q.value


def gvl_modularity(ctx, n, m, d_offsets, d_indices, d_weights, d_membership, resolution, d_workspace,
                   workspace_bytes) -> float:
    q = ctypes.c_double(0.0)
    code = load_library().gvl_modularity(ctx, n, m, d_offsets, d_indices, d_weights, d_membership, resolution,
                                         d_workspace, workspace_bytes, ctypes.byref(q))
    _check(code, "gvl_modularity")
    return q.value


def gvl_gather_probe(ctx, d_idx, n_idx, d_table, n_table, d_sink) -> None:
    """Enqueues the random-gather probe (sum of d_table[d_idx[e]] into the
    device uint64 *d_sink) on the context's stream."""
    _check(load_library().gvl_gather_probe(ctx, d_idx, n_idx, d_table, n_table, d_sink), "gvl_gather_probe")


def gvl_disconnected_communities(ctx, n, m, d_offsets, d_indices, d_membership, d_workspace, workspace_bytes,
                                 d_flags=None) -> int:
    count = ctypes.c_int64(0)
    code = load_library().gvl_disconnected_communities(ctx, n, m, d_offsets, d_indices, d_membership, d_workspace,
                                                       workspace_bytes, d_flags, ctypes.byref(count))
    _check(code, "gvl_disconnected_communities")
    return count.value


def gvl_debug_pass_info(ctx, p: int):
    n, ncom, m = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().gvl_debug_pass_info(ctx, p, ctypes.byref(n), ctypes.byref(ncom), ctypes.byref(m)),
           "gvl_debug_pass_info")
    return n.value, ncom.value, m.value


def gvl_debug_export_pass(ctx, p: int):
    n, ncom, m = gvl_debug_pass_info(ctx, p)
    bound = np.zeros(max(n, 1), np.int32)
    refined = np.zeros(max(n, 1), np.int32)
    y_off = np.zeros(ncom + 1, np.int32) if m >= 0 else None
    y_idx = np.zeros(max(m, 1), np.int32) if m >= 0 else None
    y_w = np.zeros(max(m, 1), np.float64) if m >= 0 else None
    ptr = lambda a: None if a is None else a.ctypes.data
    _check(load_library().gvl_debug_export_pass(ctx, p, ptr(bound), ptr(refined), ptr(y_off), ptr(y_idx),
                                                 ptr(y_w)), "gvl_debug_export_pass")
    if m >= 0:
        y_idx, y_w = y_idx[:m], y_w[:m]
    return bound[:n], refined[:n], y_off, y_idx, y_w


def gvl_debug_pass_movers(ctx, p: int, max_it: int = 64, max_sw: int = 64):
    mv = np.full(max_it, -1, np.int64)
    rmv = np.full(max_sw, -1, np.int64)
    _check(load_library().gvl_debug_pass_movers(ctx, p, mv.ctypes.data, max_it, rmv.ctypes.data, max_sw),
           "gvl_debug_pass_movers")
    return mv[mv >= 0].tolist(), rmv[rmv >= 0].tolist()


def gvl_batch_workspace_bytes(graphs, opt: gvl_options, lanes: int) -> int:
    arr = (gvl_graph_desc * max(len(graphs), 1))(*graphs)
    b = ctypes.c_size_t(0)
    _check(load_library().gvl_batch_workspace_bytes(len(graphs), arr, ctypes.byref(opt), lanes, ctypes.byref(b)),
           "gvl_batch_workspace_bytes")
    return int(b.value)


def gvl_leiden_batch(ctx, graphs, opt: gvl_options, lanes: int, d_workspace, workspace_bytes):
    """Returns (status, modularities[num], statuses[num]); status GVL_E_BATCH means some graphs failed."""
    num = len(graphs)
    arr = (gvl_graph_desc * max(num, 1))(*graphs)
    qs = (ctypes.c_double * max(num, 1))()
    sts = (ctypes.c_int32 * max(num, 1))()
    code = load_library().gvl_leiden_batch(ctx, num, arr, ctypes.byref(opt), lanes, d_workspace, workspace_bytes,
                                           qs, sts)
    if code not in (0, -10):
        _check(code, "gvl_leiden_batch")
    return code, list(qs)[:num], list(sts)[:num]


def gvl_fused_workspace_bytes(graphs, opt: gvl_options) -> int:
    arr = (gvl_graph_desc * max(len(graphs), 1))(*graphs)
    b = ctypes.c_size_t(0)
    _check(load_library().gvl_fused_workspace_bytes(len(graphs), arr, ctypes.byref(opt), ctypes.byref(b)),
           "gvl_fused_workspace_bytes")
    return int(b.value)


def gvl_leiden_fused(ctx, graphs, opt: gvl_options, d_workspace, workspace_bytes):
    """Returns (status, modularities[num], statuses[num]); status GVL_E_BATCH means some graphs failed."""
    num = len(graphs)
    arr = (gvl_graph_desc * max(num, 1))(*graphs)
    qs = (ctypes.c_double * max(num, 1))()
    sts = (ctypes.c_int32 * max(num, 1))()
    code = load_library().gvl_leiden_fused(ctx, num, arr, ctypes.byref(opt), d_workspace, workspace_bytes, qs, sts)
    if code not in (0, -10):
        _check(code, "gvl_leiden_fused")
    return code, list(qs)[:num], list(sts)[:num]


def gvl_server_create(device: int, lanes: int, opt: gvl_options, d_arena, arena_bytes: int):
    h = ctypes.c_void_p()
    _check(load_library().gvl_server_create(ctypes.byref(h), device, lanes, ctypes.byref(opt), d_arena, arena_bytes),
           "gvl_server_create")
    return h


def gvl_server_submit(srv, graph: gvl_graph_desc) -> int:
    t = ctypes.c_uint64(0)
    _check(load_library().gvl_server_submit(srv, ctypes.byref(graph), ctypes.byref(t)), "gvl_server_submit")
    return int(t.value)


def gvl_server_poll(srv, ticket: int) -> gvl_request_info:
    info = gvl_request_info()
    _check(load_library().gvl_server_poll(srv, ticket, ctypes.byref(info)), "gvl_server_poll")
    return info


def gvl_server_wait(srv, ticket: int, timeout_ms: int = -1) -> gvl_request_info:
    info = gvl_request_info()
    _check(load_library().gvl_server_wait(srv, ticket, timeout_ms, ctypes.byref(info)), "gvl_server_wait")
    return info


def gvl_server_cancel(srv, ticket: int) -> None:
    _check(load_library().gvl_server_cancel(srv, ticket), "gvl_server_cancel")


def gvl_server_release(srv, ticket: int) -> None:
    _check(load_library().gvl_server_release(srv, ticket), "gvl_server_release")


def gvl_server_set_batching(srv, max_batch: int, max_vertices: int) -> None:
    _check(load_library().gvl_server_set_batching(srv, max_batch, max_vertices), "gvl_server_set_batching")


def gvl_server_stats(srv) -> gvl_server_info:
    info = gvl_server_info()
    _check(load_library().gvl_server_stats(srv, ctypes.byref(info)), "gvl_server_stats")
    return info


def gvl_server_destroy(srv) -> None:
    _check(load_library().gvl_server_destroy(srv), "gvl_server_destroy")


def gvl_status_string(code: int) -> str:
    return load_library().gvl_status_string(code).decode()


# -------------------------------------------------------------- convenience ---

@dataclass
class LeidenResult:
    membership: "object"   # torch.int32 tensor on the device
    modularity: float
    stats: gvl_stats


class Leiden:
    """Owns a context and a reusable workspace on one device and stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = gvl_create(device, self.stream.cuda_stream)
        self.ws = None

    def close(self):
        if self.ctx is not None:
            gvl_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, nbytes: int):
        if self.ws is None or self.ws.numel() < nbytes:
            self.ws = self.torch.empty(max(nbytes, 256), dtype=self.torch.uint8, device=self.device)
        return self.ws

    @staticmethod
    def options(mode: int = GVL_MODE_FAST, **kw) -> gvl_options:
        o = gvl_default_options(mode)
        for k, v in kw.items():
            if not hasattr(o, k):
                raise AttributeError("gvl_options has no field %r" % k)
            setattr(o, k, v)
        return o

    def run(self, offsets, indices, weights=None, resolution: float = 1.0, opt: Optional[gvl_options] = None,
            membership=None) -> LeidenResult:
        torch = self.torch
        opt = opt if opt is not None else self.options()
        n = offsets.numel() - 1
        m = indices.numel()
        for t, dt in ((offsets, torch.int32), (indices, torch.int32)):
            if t.dtype != dt or t.device != self.device or not t.is_contiguous():
                raise ValueError("offsets/indices must be contiguous int32 tensors on %s" % self.device)
        if weights is not None and (weights.dtype != torch.float32 or weights.device != self.device
                                    or not weights.is_contiguous() or weights.numel() != m):
            raise ValueError("weights must be a contiguous float32 tensor of length m on %s" % self.device)
        wsb = gvl_workspace_bytes(n, m, opt)
        ws = self.workspace(wsb)
        if membership is None:
            membership = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        st = gvl_stats()
        q = gvl_leiden(self.ctx, n, m, offsets.data_ptr(), indices.data_ptr(),
                       None if weights is None else weights.data_ptr(), float(resolution), opt,
                       ws.data_ptr(), ws.numel(), membership.data_ptr(), st)
        return LeidenResult(membership[:n], q, st)

    def modularity(self, offsets, indices, weights, membership, resolution: float = 1.0) -> float:
        n = offsets.numel() - 1
        m = indices.numel()
        opt = self.options()
        ws = self.workspace(gvl_workspace_bytes(n, m, opt))
        return gvl_modularity(self.ctx, n, m, offsets.data_ptr(), indices.data_ptr(),
                              None if weights is None else weights.data_ptr(), membership.data_ptr(),
                              float(resolution), ws.data_ptr(), ws.numel())

    def disconnected(self, offsets, indices, membership, flags=None) -> int:
        """Alg. 5 on the device: communities of `membership` that are not connected."""
        n = offsets.numel() - 1
        m = indices.numel()
        ws = self.workspace(gvl_workspace_bytes(n, m, self.options()))
        return gvl_disconnected_communities(self.ctx, n, m, offsets.data_ptr(),
                                            indices.data_ptr() if m else None, membership.data_ptr(),
                                            ws.data_ptr(), ws.numel(), None if flags is None else flags.data_ptr())


def leiden(offsets, indices, weights=None, resolution: float = 1.0, mode: int = GVL_MODE_FAST, **kw):
    """One-shot Leiden on device tensors; returns (membership, modularity, stats)."""
    eng = Leiden(offsets.device.index or 0)
    try:
        r = eng.run(offsets, indices, weights, resolution, eng.options(mode, **kw))
        return r.membership, r.modularity, r.stats
    finally:
        eng.close()


def graph_desc(offsets, indices, weights, membership, resolution: float = 1.0) -> gvl_graph_desc:
    """Descriptor of one graph held in device tensors (int32 offsets/indices, float32 weights or None)."""
    return gvl_graph_desc(offsets.numel() - 1, indices.numel(), offsets.data_ptr(),
                          indices.data_ptr() if indices.numel() else None,
                          None if weights is None else weights.data_ptr(), float(resolution),
                          None if membership is None else membership.data_ptr())


class Server:
    """Continuous-batching Leiden server over a device arena (a torch uint8
    tensor) that holds the workspaces of running requests.

    Inputs must be fully written before ``submit`` (synchronise the stream
    that produced them); the membership tensor is complete once ``wait``
    or ``poll`` reports GVL_REQ_DONE.
    """

    def __init__(self, arena, lanes: int = 4, opt: Optional[gvl_options] = None):
        self.arena = arena
        opt = opt if opt is not None else Leiden.options()
        self.srv = gvl_server_create(arena.device.index or 0, lanes, opt, arena.data_ptr(), arena.numel())

    def submit(self, offsets, indices, weights, membership, resolution: float = 1.0) -> int:
        return gvl_server_submit(self.srv, graph_desc(offsets, indices, weights, membership, resolution))

    def poll(self, ticket: int) -> gvl_request_info:
        return gvl_server_poll(self.srv, ticket)

    def wait(self, ticket: int, timeout_ms: int = -1) -> gvl_request_info:
        return gvl_server_wait(self.srv, ticket, timeout_ms)

    def cancel(self, ticket: int) -> None:
        gvl_server_cancel(self.srv, ticket)

    def release(self, ticket: int) -> None:
        gvl_server_release(self.srv, ticket)

    def set_batching(self, max_batch: int, max_vertices: int) -> None:
        gvl_server_set_batching(self.srv, max_batch, max_vertices)

    def stats(self) -> gvl_server_info:
        return gvl_server_stats(self.srv)

    def close(self) -> None:
        if self.srv is not None:
            gvl_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
