"""A giant community whose super-vertex row outgrows the partition tables.

Alg. 4 writes one row per community.  Giant communities (more than 8192
member arcs) are aggregated by key partitions, at most 256 of them, each
summed in an LDS table; when a partition holds more distinct neighbour
communities than its table, it emits its share of the row in several parts,
so the row may list a neighbour more than once with partial weights.  The
graph here forces that case: a 1100-vertex clique of weight-10 edges (one
refined community of 4.4M member arcs) and 1.6M weight-50 pairs, each
member of a pair linked by a unit edge to a different clique vertex (1.6M
distinct neighbour communities, each seen from two member rows: about 6250
keys per partition, above the 6144 slots of a partition table).
Deterministic mode must still match the oracle bit for bit, and the merged
row must equal the oracle's.
"""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2312_13936_amd as gvl  # noqa: E402
from test_gpu_parity import FAST_TOL, run  # noqa: E402

CORE, PAIRS = 1100, 1600000


def core_and_pairs():
    iu = np.triu_indices(CORE, 1)
    core = np.stack([iu[0], iu[1]], 1)
    a = CORE + 2 * np.arange(PAIRS)
    pairs = np.stack([a, a + 1], 1)
    q = np.arange(PAIRS)
    links = np.concatenate([np.stack([a, q % CORE], 1), np.stack([a + 1, (q + CORE // 2) % CORE], 1)])
    edges = np.concatenate([core, pairs, links]).astype(np.int32)
    w = np.concatenate([np.full(len(core), 10.0), np.full(PAIRS, 50.0), np.ones(2 * PAIRS)]).astype(np.float32)
    return gen.from_edges(CORE + 2 * PAIRS, edges, w, name="clique+pairs")


@pytest.fixture(scope="module")
def eng():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    e = gvl.Leiden(0)
    yield e
    e.close()


@pytest.fixture(scope="module")
def g():
    return core_and_pairs()


def merged(off, idx, w, r):
    a, b = int(off[r]), int(off[r + 1])
    keys, inv = np.unique(idx[a:b], return_inverse=True)
    return keys, np.bincount(inv, weights=w[a:b])


def test_giant_row_in_parts_det_bit_exact(eng, g):
    print("giant row det:", g.n, g.m, flush=True)
    mem, q, st = run(eng, g, gvl.GVL_MODE_DET, debug_trace=1)
    o = oracle.leiden(g, mode=oracle.DET_SYNC, trace=True)
    assert np.array_equal(mem, o.membership)
    assert q == o.q
    assert st.passes == len(o.passes)
    # pass 0: the clique is one refined community; its row, merged, is the oracle's
    _, refined, y_off, y_idx, y_w = gvl.gvl_debug_export_pass(eng.ctx, 0)
    t = o.passes[0]
    assert np.array_equal(refined, t.refined)
    used = np.unique(t.refined)
    big = int(np.searchsorted(used, t.refined[0]))  # super-vertex of the clique
    ok, ow = t.y_idx[t.y_off[big]:t.y_off[big + 1]], t.y_w[t.y_off[big]:t.y_off[big + 1]]
    assert len(ok) == PAIRS + 1
    gk, gw = merged(y_off, y_idx, y_w, big)
    assert np.array_equal(gk, ok) and np.array_equal(gw, ow)
    # the row was emitted in parts (a neighbour listed more than once)
    assert y_off[big + 1] - y_off[big] > len(ok)
    # every other row is exactly the oracle's
    assert len(y_off) == len(t.y_off)
    glen, olen = np.diff(y_off), np.diff(t.y_off)
    glen[big] = olen[big] = 0
    assert np.array_equal(glen, olen)
    cut = lambda a, off: np.concatenate([a[:off[big]], a[off[big + 1]:]])
    assert np.array_equal(cut(y_idx, y_off), cut(t.y_idx, t.y_off))
    assert np.array_equal(cut(y_w, y_off), cut(t.y_w, t.y_off))


def test_giant_row_in_parts_fast_quality(eng, g):
    print("giant row fast:", g.n, g.m, flush=True)
    mem, q, st = run(eng, g, gvl.GVL_MODE_FAST)
    assert q == oracle.modularity(g, mem)
    assert oracle.disconnected(g, mem) == 0
    qref = min(oracle.leiden(g, mode=oracle.SEQ_ASYNC).q, oracle.leiden(g, mode=oracle.DET_SYNC).q)
    assert q >= qref - FAST_TOL
