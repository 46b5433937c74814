"""The seeded input generators keep the promises of the input recipe.

Every graph the tests and the benchmark use comes from `gen`: symmetric
CSR, no self-loops (except where an edge list asks for one) and no
duplicate arcs, the degree and weight structure the recipe names, and the
same graph for the same seed.  These run on the CPU.
"""
import numpy as np
import pytest

import gen


def arcs(g):
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.offsets.astype(np.int64)))
    return src, g.indices.astype(np.int64), g.weights.astype(np.float64)


def check_csr(g, self_loops=False):
    off = g.offsets.astype(np.int64)
    assert off[0] == 0 and off[-1] == g.m and np.all(np.diff(off) >= 0)
    src, dst, w = arcs(g)
    assert np.all((dst >= 0) & (dst < g.n))
    if not self_loops:
        assert not np.any(src == dst)
    key = src * g.n + dst
    assert len(np.unique(key)) == g.m, "duplicate arcs"
    # symmetric with equal weights
    order = np.argsort(key)
    rev = dst * g.n + src
    pos = np.searchsorted(key[order], rev)
    assert np.all(pos < g.m) and np.array_equal(key[order][pos], rev)
    assert np.array_equal(w[order][pos], w)
    assert np.all(w > 0)


def same(g1, g2):
    return (g1.n == g2.n and np.array_equal(g1.offsets, g2.offsets) and np.array_equal(g1.indices, g2.indices)
            and np.array_equal(g1.weights, g2.weights))


def test_rmat_is_a_simple_symmetric_unit_graph_with_hubs():
    g = gen.rmat(14, 16, 0.57, 0.19, 0.19, seed=2)
    check_csr(g)
    assert g.n == 1 << 14
    assert np.all(g.weights == 1.0)
    deg = np.diff(g.offsets)
    # 2 * 16 * 2^14 samples before symmetrisation and dedup
    assert 0.6 * 2 * 16 * g.n < g.m <= 2 * 16 * g.n
    # skewed: the top 1 % of vertices hold a large share of the arcs, and some have none
    top = np.sort(deg)[::-1][: g.n // 100].sum()
    assert top > 0.15 * g.m
    assert np.any(deg == 0)
    assert same(g, gen.rmat(14, 16, 0.57, 0.19, 0.19, seed=2))
    assert not same(g, gen.rmat(14, 16, 0.57, 0.19, 0.19, seed=3))


def test_planted_partition_densities():
    blocks, size, p_in, p_out = 10, 300, 0.05, 0.002
    g = gen.planted(blocks, size, p_in, p_out, seed=4)
    check_csr(g)
    assert g.truth is not None and np.array_equal(np.bincount(g.truth), np.full(blocks, size))
    src, dst, _ = arcs(g)
    intra = int(np.sum(g.truth[src] == g.truth[dst])) // 2
    inter = g.m // 2 - intra
    e_intra = blocks * size * (size - 1) / 2 * p_in
    e_inter = blocks * (blocks - 1) / 2 * size * size * p_out
    assert abs(intra - e_intra) < 5 * np.sqrt(e_intra)
    assert abs(inter - e_inter) < 5 * np.sqrt(e_inter)
    assert same(g, gen.planted(blocks, size, p_in, p_out, seed=4))


def test_grid_degrees_and_integer_weights():
    rows, cols = 64, 48
    g = gen.grid(rows, cols, drop=0.1, diag_frac=0.01, wmax=100, seed=5)
    check_csr(g)
    assert g.n == rows * cols
    deg = np.diff(g.offsets)
    assert deg.max() <= 8
    w = g.weights
    assert np.all(w == np.floor(w)) and w.min() >= 1 and w.max() <= 100
    # about 90 % of the 2 r c - r - c lattice edges survive, plus 1 % diagonals
    lattice = 2 * rows * cols - rows - cols
    assert 0.8 * lattice < g.m // 2 < 1.0 * lattice + 0.02 * rows * cols


def test_lfr_degrees_and_mixing():
    g = gen.lfr(20000, avg_deg=12.0, mu=0.3, seed=7)
    check_csr(g)
    assert np.all(g.weights == 1.0)
    deg = np.diff(g.offsets)
    # the requested mean: stubs that would form self-loops or repeat an edge
    # are paired again, so only a few per cent stay unpaired
    assert 0.95 * 12.0 < deg.mean() <= 1.02 * 12.0
    for n, k in ((2000, 12.0), (200000, 12.0), (300000, 16.0)):
        d = np.diff(gen.lfr(n, avg_deg=k, mu=0.3, seed=3).offsets)
        assert 0.95 * k < d.mean() <= 1.02 * k, (n, k, d.mean())
    assert deg.max() > 4 * deg.mean()  # power-law tail
    src, dst, _ = arcs(g)
    mixing = np.mean(g.truth[src] != g.truth[dst])
    assert 0.2 < mixing < 0.4
    assert same(g, gen.lfr(20000, avg_deg=12.0, mu=0.3, seed=7))


def test_from_edges_sums_duplicates_and_keeps_one_self_loop():
    g = gen.from_edges(4, [(0, 1), (1, 0), (2, 2), (2, 3)], [1.0, 2.0, 5.0, 1.0])
    check_csr(g, self_loops=True)
    src, dst, w = arcs(g)
    d = {(int(a), int(b)): float(x) for a, b, x in zip(src, dst, w)}
    assert d[(0, 1)] == 3.0 and d[(1, 0)] == 3.0
    assert d[(2, 2)] == 5.0 and sum(1 for a, b in d if a == b) == 1
    assert d[(2, 3)] == 1.0 and d[(3, 2)] == 1.0


@pytest.mark.parametrize("seed", [1, 2])
def test_lfr_sizes_are_log_uniform_in_range(seed):
    s = gen.lfr_sizes(4096, 1000, 200000, seed)
    assert s.min() >= 1000 and s.max() <= 200000
    # log-uniform: the median sits near the geometric mean of the ends
    assert abs(np.log(np.median(s)) - 0.5 * (np.log(1000) + np.log(200000))) < 0.15
