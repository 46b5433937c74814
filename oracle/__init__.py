"""CPU oracle for GVE-Leiden (ctypes wrapper around ``oracle.cpp``).

TEST INFRASTRUCTURE ONLY: only the tests, the graft smoke check and the
benchmark's CPU-baseline leg may import this module.  The product path
(``paper_2312_13936_amd``) never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

SEQ_ASYNC = 0
DET_SYNC = 1


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (single-threaded, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("tolerance", ctypes.c_double),
                ("tolerance_drop", ctypes.c_double), ("aggregation_tolerance", ctypes.c_double),
                ("max_iterations", ctypes.c_int32), ("max_passes", ctypes.c_int32),
                ("refine_sweeps", ctypes.c_int32), ("subsweeps", ctypes.c_int32),
                ("resolution", ctypes.c_double), ("trace", ctypes.c_int32), ("louvain", ctypes.c_int32),
                ("refine_random", ctypes.c_int32), ("seed", ctypes.c_uint32),
                ("shrink_excludes_isolated", ctypes.c_int32), ("refine_based", ctypes.c_int32)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.oracle_default_opts.argtypes = [ctypes.POINTER(Opts), i32]
        lib.oracle_default_opts.restype = None
        lib.oracle_leiden.argtypes = [i64, vp, vp, vp, ctypes.POINTER(Opts), ctypes.POINTER(i32)]
        lib.oracle_leiden.restype = vp
        lib.oracle_free.argtypes = [vp]
        lib.oracle_free.restype = None
        lib.oracle_result.argtypes = [vp, vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        lib.oracle_result.restype = dbl
        lib.oracle_pass_info.argtypes = [vp, i32, vp]
        lib.oracle_pass_info.restype = ctypes.c_int
        lib.oracle_pass_movers.argtypes = [vp, i32, vp, vp]
        lib.oracle_pass_movers.restype = ctypes.c_int
        lib.oracle_pass_get.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        lib.oracle_pass_get.restype = ctypes.c_int
        lib.oracle_modularity.argtypes = [i64, vp, vp, vp, vp, dbl]
        lib.oracle_modularity.restype = dbl
        lib.oracle_delta_modularity.argtypes = [i64, vp, vp, vp, vp, i64, i32, dbl]
        lib.oracle_delta_modularity.restype = dbl
        lib.oracle_aggregate.argtypes = [i64, vp, vp, vp, vp, i64, vp, vp, vp]
        lib.oracle_aggregate.restype = i64
        lib.oracle_random_score.argtypes = [dbl, ctypes.c_uint32, i32, i32, i64, i32]
        lib.oracle_random_score.restype = dbl
        lib.oracle_neg_ln_unit.argtypes = [ctypes.c_uint32]
        lib.oracle_neg_ln_unit.restype = dbl
        lib.oracle_disconnected.argtypes = [i64, vp, vp, vp, vp]
        lib.oracle_disconnected.restype = i64
        lib.oracle_gain_key.argtypes = [i64, i64, i64, i64, i64, i64, i64, ctypes.POINTER(i64),
                                        ctypes.POINTER(ctypes.c_uint64)]
        lib.oracle_gain_key.restype = None
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _csr(g):
    off = np.ascontiguousarray(g.offsets, dtype=np.int32)
    idx = np.ascontiguousarray(g.indices, dtype=np.int32)
    w = None if g.weights is None else np.ascontiguousarray(g.weights, dtype=np.float32)
    return off, idx, w


@dataclass
class PassTrace:
    n: int
    m: int
    iterations: int
    converged_first: int
    refine_sweeps: int
    communities: int
    movers: List[int]
    refine_movers: List[int]
    bound: Optional[np.ndarray] = None
    refined: Optional[np.ndarray] = None
    y_off: Optional[np.ndarray] = None
    y_idx: Optional[np.ndarray] = None
    y_w: Optional[np.ndarray] = None


@dataclass
class Result:
    membership: np.ndarray
    q: float
    termination: int
    passes: List[PassTrace] = field(default_factory=list)


def default_opts(mode: int = SEQ_ASYNC) -> Opts:
    o = Opts()
    _load().oracle_default_opts(ctypes.byref(o), mode)
    return o


def leiden(g, mode: int = SEQ_ASYNC, resolution: float = 1.0, trace: bool = False, **kw) -> Result:
    """Run the oracle on a gen.Graph-like object (n, offsets, indices, weights)."""
    lib = _load()
    o = default_opts(mode)
    o.resolution = resolution
    o.trace = 1 if trace else 0
    for k, v in kw.items():
        setattr(o, k, v)
    off, idx, w = _csr(g)
    st = ctypes.c_int32(0)
    h = lib.oracle_leiden(g.n, _p(off), _p(idx), _p(w), ctypes.byref(o), ctypes.byref(st))
    if not h:
        raise ValueError("oracle_leiden rejected the input (status %d)" % st.value)
    try:
        mem = np.zeros(g.n, np.int32)
        npass = ctypes.c_int32(0)
        term = ctypes.c_int32(0)
        q = lib.oracle_result(h, _p(mem), ctypes.byref(npass), ctypes.byref(term))
        res = Result(mem, q, term.value)
        info = np.zeros(8, np.int64)
        for p in range(npass.value):
            lib.oracle_pass_info(h, p, _p(info))
            n, m, it, first, rs, ncom, ym, agg = [int(x) for x in info]
            mv = np.zeros(max(it, 1), np.int64)
            rmv = np.zeros(max(rs, 1), np.int64)
            lib.oracle_pass_movers(h, p, _p(mv), _p(rmv))
            t = PassTrace(n, m, it, first, rs, ncom, mv[:it].tolist(), rmv[:rs].tolist())
            if trace:
                t.bound = np.zeros(n, np.int32)
                t.refined = np.zeros(n, np.int32)
                if agg:
                    t.y_off = np.zeros(ncom + 1, np.int32)
                    t.y_idx = np.zeros(max(ym, 1), np.int32)
                    t.y_w = np.zeros(max(ym, 1), np.float64)
                lib.oracle_pass_get(h, p, _p(t.bound), _p(t.refined), _p(t.y_off), _p(t.y_idx), _p(t.y_w))
                if agg:
                    t.y_idx = t.y_idx[:ym]
                    t.y_w = t.y_w[:ym]
            res.passes.append(t)
        return res
    finally:
        lib.oracle_free(h)


def modularity(g, membership, resolution: float = 1.0) -> float:
    """Eq. 1 (exact integer sums when the weights are integral)."""
    off, idx, w = _csr(g)
    mem = np.ascontiguousarray(membership, dtype=np.int32)
    return _load().oracle_modularity(g.n, _p(off), _p(idx), _p(w), _p(mem), resolution)


def delta_modularity(g, membership, i: int, c: int, resolution: float = 1.0) -> float:
    """Eq. 2: gain of moving vertex i from its community to community c (FP64)."""
    off, idx, w = _csr(g)
    mem = np.ascontiguousarray(membership, dtype=np.int32)
    return _load().oracle_delta_modularity(g.n, _p(off), _p(idx), _p(w), _p(mem), i, c, resolution)


def aggregate(g, labels, nc: int):
    """Alg. 4: canonical super-vertex CSR (offsets, indices, float64 weights)."""
    lib = _load()
    off, idx, w = _csr(g)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    m = lib.oracle_aggregate(g.n, _p(off), _p(idx), _p(w), _p(lab), nc, None, None, None)
    y_off = np.zeros(nc + 1, np.int32)
    y_idx = np.zeros(max(m, 1), np.int32)
    y_w = np.zeros(max(m, 1), np.float64)
    lib.oracle_aggregate(g.n, _p(off), _p(idx), _p(w), _p(lab), nc, _p(y_off), _p(y_idx), _p(y_w))
    return y_off, y_idx[:m], y_w[:m]


def disconnected(g, membership) -> int:
    """Alg. 5: number of communities whose members are not connected inside the community."""
    off, idx, _ = _csr(g)
    mem = np.ascontiguousarray(membership, dtype=np.int32)
    flags = np.zeros(g.n, np.int32)
    return int(_load().oracle_disconnected(g.n, _p(off), _p(idx), _p(mem), _p(flags)))


def random_score(gain: float, seed: int, pass_: int, sweep: int, i: int, c: int) -> float:
    """Randomized refinement: selection score gain / (-ln u) of candidate c."""
    return float(_load().oracle_random_score(gain, seed, pass_, sweep, i, c))


def neg_ln_unit(x: int) -> float:
    """-ln((x + 1/2) / 2^32) as the randomized refinement computes it."""
    return float(_load().oracle_neg_ln_unit(x))


def gain_key(kic: int, kid: int, ki: int, sc: int, sd: int, W: int, p: int) -> int:
    """The deterministic mode's exact Eq. 2 key for gamma = p / 2^16, as a Python int."""
    hi = ctypes.c_int64(0)
    lo = ctypes.c_uint64(0)
    _load().oracle_gain_key(kic, kid, ki, sc, sd, W, p, ctypes.byref(hi), ctypes.byref(lo))
    return (hi.value << 64) | lo.value
