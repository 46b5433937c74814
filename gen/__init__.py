"""Seeded synthetic graph generators shared by the oracle tests, the GPU tests
and the benchmark.

This module only produces inputs (CSR arrays); it holds none of the
community-detection arithmetic.  The generators live in ``gen.cpp`` and are
built into ``libgen.so`` next to this file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.cpp")
_LIB_PATH = os.path.join(_HERE, "libgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile libgen.so (g++, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _GenGraph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64),
                ("offsets", ctypes.POINTER(ctypes.c_int32)),
                ("indices", ctypes.POINTER(ctypes.c_int32)),
                ("weights", ctypes.POINTER(ctypes.c_float)),
                ("truth", ctypes.POINTER(ctypes.c_int32))]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(_GenGraph)
        lib.gen_free.argtypes = [P]
        lib.gen_planted.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_uint64, P]
        lib.gen_rmat.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_uint64, P]
        lib.gen_grid.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int32, ctypes.c_uint64, P]
        lib.gen_from_edges.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, P]
        lib.gen_lfr.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, P]
        for f in (lib.gen_planted, lib.gen_rmat, lib.gen_grid, lib.gen_from_edges, lib.gen_lfr):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class Graph:
    """Symmetric CSR graph: int32 offsets[n+1], int32 indices[m], float32 weights[m]."""
    n: int
    m: int
    offsets: np.ndarray
    indices: np.ndarray
    weights: np.ndarray
    truth: Optional[np.ndarray] = None
    name: str = ""


def _take(g: _GenGraph, lib, name: str) -> Graph:
    n, m = int(g.n), int(g.m)
    off = np.ctypeslib.as_array(g.offsets, shape=(n + 1,)).copy()
    if m > 0:
        idx = np.ctypeslib.as_array(g.indices, shape=(m,)).copy()
        wt = np.ctypeslib.as_array(g.weights, shape=(m,)).copy()
    else:
        idx = np.zeros(0, np.int32)
        wt = np.zeros(0, np.float32)
    truth = np.ctypeslib.as_array(g.truth, shape=(n,)).copy() if bool(g.truth) else None
    lib.gen_free(ctypes.byref(g))
    return Graph(n, m, off, idx, wt, truth, name)


def _call(fn, args, name):
    lib = _load()
    g = _GenGraph()
    rc = getattr(lib, fn)(*args, ctypes.byref(g))
    if rc != 0:
        lib.gen_free(ctypes.byref(g))
        raise RuntimeError("%s failed with code %d" % (fn, rc))
    return _take(g, lib, name)


def planted(blocks: int = 20, block_size: int = 500, p_in: float = 0.02, p_out: float = 0.0005,
            seed: int = 1) -> Graph:
    """Stochastic block model with equal blocks, ids shuffled (truth = block)."""
    return _call("gen_planted", (blocks, block_size, p_in, p_out, seed),
                 "planted-%dx%d" % (blocks, block_size))


def rmat(scale: int = 24, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 2) -> Graph:
    """R-MAT graph, symmetrised, self-loops and duplicates removed, ids shuffled."""
    return _call("gen_rmat", (scale, edge_factor, a, b, c, seed), "rmat-s%d-ef%d" % (scale, edge_factor))


def grid(rows: int = 4096, cols: int = 4096, drop: float = 0.1, diag_frac: float = 0.01,
         wmax: int = 100, seed: int = 3) -> Graph:
    """Lattice with dropped edges, diagonal shortcuts and integer weights in [1, wmax]."""
    return _call("gen_grid", (rows, cols, drop, diag_frac, wmax, seed), "grid-%dx%d" % (rows, cols))


def lfr(n: int, avg_deg: float = 12.0, tau1: float = 2.5, tau2: float = 1.5, mu: float = 0.3,
        kmax: int = 0, cmin: int = 20, cmax: int = 0, seed: int = 1000) -> Graph:
    """LFR-style graph: power-law degrees and community sizes, mixing mu,
    unit weights (truth = planted community).  Defaults: kmax = min(4 sqrt(n),
    n/10), community sizes on [20, max(20, n/10)]."""
    if kmax <= 0:
        kmax = max(2, min(int(4 * n ** 0.5), n // 10))
    if cmax <= 0:
        cmax = max(cmin, n // 10)
    return _call("gen_lfr", (n, avg_deg, kmax, tau1, tau2, mu, cmin, cmax, seed), "lfr-%d-%d" % (n, seed))


def lfr_sizes(count: int, lo: int, hi: int, seed: int):
    """Vertex counts log-uniform on [lo, hi] (seeded)."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(lo), np.log(hi), count)).astype(np.int64)


def from_edges(n: int, edges, weights=None, name: str = "edges") -> Graph:
    """Symmetric CSR from an undirected edge list; self-loops stored once, duplicates summed."""
    e = np.asarray(edges, dtype=np.int32).reshape(-1, 2)
    us = np.ascontiguousarray(e[:, 0])
    vs = np.ascontiguousarray(e[:, 1])
    ws = None if weights is None else np.ascontiguousarray(np.asarray(weights, dtype=np.float32))
    return _call("gen_from_edges", (n, len(us), us.ctypes.data, vs.ctypes.data,
                                    None if ws is None else ws.ctypes.data), name)


# ----- small structured graphs used by the tests -------------------------------------------

def clique_edges(nodes):
    nodes = list(nodes)
    return [(nodes[a], nodes[b]) for a in range(len(nodes)) for b in range(a + 1, len(nodes))]


def ring_of_cliques(k: int, s: int) -> Graph:
    """k cliques K_s joined in a ring by one edge between consecutive cliques."""
    edges = []
    for q in range(k):
        edges += clique_edges(range(q * s, (q + 1) * s))
        edges.append((q * s, ((q + 1) % k) * s + 1 if s > 1 else ((q + 1) % k) * s))
    return from_edges(k * s, edges, name="ring-%dxK%d" % (k, s))


def cliques_with_bridge(s: int) -> Graph:
    """Two K_s joined by a single edge."""
    edges = clique_edges(range(s)) + clique_edges(range(s, 2 * s)) + [(0, s)]
    return from_edges(2 * s, edges, name="2xK%d+bridge" % s)


def random_graph(n: int, p: float, seed: int, wmax: int = 1, self_loops: bool = False) -> Graph:
    """Small Erdos-Renyi graph with integer weights in [1, wmax] (test inputs)."""
    rng = np.random.default_rng(seed)
    edges, ws = [], []
    for u in range(n):
        for v in range(u if self_loops else u + 1, n):
            if rng.random() < p:
                edges.append((u, v))
                ws.append(float(rng.integers(1, wmax + 1)))
    if not edges:
        return Graph(n, 0, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32),
                     None, "empty")
    return from_edges(n, edges, ws, name="er-%d-%g-%d" % (n, p, seed))
