"""GPU parity of the Louvain mode (no refinement) and of the device-side
disconnected-community check (Alg. 5), both against the CPU oracle.

Deterministic Louvain must match the oracle's det-sync Louvain bit for bit
(membership, modularity, per-pass labels and super-vertex CSRs); the device
check must report the same number of disconnected communities, and flag the
same labels, as the oracle's breadth-first search.
"""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2312_13936_amd as gvl  # noqa: E402
from test_gpu_parity import GRAPHS, dev, graph, run  # noqa: E402


@pytest.fixture(scope="module")
def eng():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    e = gvl.Leiden(0)
    yield e
    e.close()


def check(eng, g, mem):
    off, idx, _ = dev(g)
    m = torch.from_numpy(np.ascontiguousarray(mem, dtype=np.int32)).to("cuda")
    flags = torch.full((max(g.n, 1),), -3, dtype=torch.int32, device="cuda")
    count = eng.disconnected(off, idx, m, flags)
    torch.cuda.synchronize()
    return count, flags[:g.n].cpu().numpy()


def oracle_check(g, mem):
    f = np.zeros(max(g.n, 1), np.int32)
    from oracle import _load, _p, _csr
    off, idx, _ = _csr(g)
    cnt = _load().oracle_disconnected(g.n, _p(off), _p(idx), _p(np.ascontiguousarray(mem, np.int32)), _p(f))
    return int(cnt), f[:g.n]


def assert_same_check(eng, g, mem, what):
    c, f = check(eng, g, mem)
    oc, of = oracle_check(g, mem)
    assert c == oc, (what, c, oc)
    assert np.array_equal(f, of), what


@pytest.mark.parametrize("name", ["rmat-s14", "grid200-w100", "er-selfloops", "hubs-wide", "star", "path"])
def test_disconnected_random_labels(eng, name):
    g = graph(name)
    rng = np.random.default_rng(5)
    for k in (1, 3, 50, max(2, g.n // 4)):
        mem = rng.integers(0, k, g.n).astype(np.int32)
        print("check:", name, "labels", k, flush=True)
        assert_same_check(eng, g, mem, (name, k))


@pytest.mark.parametrize("name", ["rmat-s12", "rmat-s14", "planted-small", "grid64-w100"])
def test_disconnected_of_results(eng, name):
    g = graph(name)
    for mode in (gvl.GVL_MODE_DET, gvl.GVL_MODE_FAST):
        lei, _, _ = run(eng, g, mode)
        c, _ = check(eng, g, lei)
        assert c == 0, (name, mode)  # Leiden: every community connected
        lou, _, _ = run(eng, g, mode, louvain=1)
        assert_same_check(eng, g, lou, (name, mode, "louvain"))


def test_disconnected_edge_cases(eng):
    # every vertex its own community; one community over isolated vertices;
    # no arcs at all
    g = gen.from_edges(6, [(0, 1), (1, 2), (3, 4)])
    assert_same_check(eng, g, np.arange(6, dtype=np.int32), "singletons")
    assert_same_check(eng, g, np.zeros(6, np.int32), "one community")  # {0,1,2}, {3,4}, {5}: disconnected
    assert check(eng, g, np.zeros(6, np.int32))[0] == 1
    assert_same_check(eng, g, np.array([0, 0, 0, 1, 1, 2], np.int32), "components")
    e = gen.Graph(4, 0, np.zeros(5, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    assert_same_check(eng, e, np.array([0, 0, 1, 1], np.int32), "edgeless")


def test_disconnected_full_size_random_labels(eng):
    # R-MAT scale 16, labels drawn so that most communities are split
    g = graph("rmat-s16")
    mem = np.random.default_rng(9).integers(0, 5000, g.n).astype(np.int32)
    assert_same_check(eng, g, mem, "rmat-s16")


LOUVAIN_GRAPHS = ["ring10xK5", "ring30xK3", "planted-small", "grid64-w100", "rmat-s12", "rmat-s14",
                  "er-selfloops", "hub+cliques", "hubs-wide"]


@pytest.mark.parametrize("name", LOUVAIN_GRAPHS)
def test_louvain_det_bit_exact(eng, name):
    g = graph(name)
    print("louvain det parity:", name, flush=True)
    mem, q, st = run(eng, g, gvl.GVL_MODE_DET, louvain=1, debug_trace=1)
    o = oracle.leiden(g, mode=oracle.DET_SYNC, louvain=1, trace=True)
    assert st.passes == len(o.passes)
    for p, t in enumerate(o.passes):
        bound, refined, y_off, y_idx, y_w = gvl.gvl_debug_export_pass(eng.ctx, p)
        assert np.array_equal(bound, t.bound), "pass %d bound labels" % p
        assert np.array_equal(refined, t.bound), "pass %d: no refinement" % p
        if t.y_off is not None:
            assert np.array_equal(y_off, t.y_off) and np.array_equal(y_idx, t.y_idx), p
            assert np.array_equal(y_w, t.y_w), p
    assert np.array_equal(mem, o.membership)
    assert q == o.q
    assert st.termination == o.termination


# Per-graph margin wider than 1e-3, by rule (i) of test_gpu_parity.py:
#   rmat-s14  the sequential Louvain oracle's spread over the given and seven
#             seeded numberings is 3.07e-3 (0.100831 .. 0.103904); its
#             group-synchronous run (exact arithmetic) lands 2.45e-3 below
#             the given numbering's sequential result
LOUVAIN_WIDER = {"rmat-s14": 3.1e-3}


@pytest.mark.parametrize("name", ["rmat-s14", "planted-C1", "grid200-w100", "hubs-wide"])
def test_louvain_fast_quality(eng, name):
    g = graph(name)
    mem, q, _ = run(eng, g, gvl.GVL_MODE_FAST, louvain=1)
    assert q == oracle.modularity(g, mem)  # reported Q is Eq. 1 of the returned membership
    # the fast-mode bar: the sequential oracle (Louvain too) on the graph as
    # numbered, minus 1e-3 (or LOUVAIN_WIDER's margin)
    ref = oracle.leiden(g, mode=oracle.SEQ_ASYNC, louvain=1).q
    print("  louvain %s: fast Q %.6f, sequential oracle %.6f, margin %+.6f" % (name, q, ref, q - ref), flush=True)
    assert q >= ref - LOUVAIN_WIDER.get(name, 1e-3), (q, ref)


def test_louvain_fused_matches_solo(eng):
    from test_gpu_batch_serve import run_fused
    gs = [graph(k) for k in ("rmat-s12", "planted-small", "hub+cliques", "grid64-w100")]
    code, mems, qs, sts = run_fused(eng, gs, gvl.GVL_MODE_DET, louvain=1)
    assert code == 0 and all(x == 0 for x in sts)
    for g, mem, q in zip(gs, mems, qs):
        o = oracle.leiden(g, mode=oracle.DET_SYNC, louvain=1)
        assert np.array_equal(mem, o.membership) and q == o.q, g.name


# ------------------------------------------------ randomized refinement ---

RANDOM_GRAPHS = ["ring30xK3", "planted-small", "grid64-w100", "rmat-s12", "rmat-s14", "er-selfloops",
                 "hub+cliques", "hubs-wide"]


@pytest.mark.parametrize("seed", [1, 12345])
@pytest.mark.parametrize("name", RANDOM_GRAPHS)
def test_random_refinement_det_bit_exact(eng, name, seed):
    g = graph(name)
    print("random refinement det parity:", name, seed, flush=True)
    mem, q, st = run(eng, g, gvl.GVL_MODE_DET, refine_random=1, seed=seed, debug_trace=1)
    o = oracle.leiden(g, mode=oracle.DET_SYNC, refine_random=1, seed=seed, trace=True)
    assert st.passes == len(o.passes)
    for p, t in enumerate(o.passes):
        bound, refined, _, _, _ = gvl.gvl_debug_export_pass(eng.ctx, p)
        movers, rmovers = gvl.gvl_debug_pass_movers(eng.ctx, p)
        assert rmovers == t.refine_movers, "pass %d refinement movers" % p
        assert np.array_equal(bound, t.bound), "pass %d bound labels" % p
        assert np.array_equal(refined, t.refined), "pass %d refined labels" % p
    assert np.array_equal(mem, o.membership)
    assert q == o.q
    c, _ = check(eng, g, mem)
    assert c == 0


def test_random_refinement_fused_matches_oracle(eng):
    # draws use graph-local vertex and community ids, so a graph's result
    # does not depend on its place in the union
    from test_gpu_batch_serve import run_fused
    gs = [graph(k) for k in ("rmat-s12", "planted-small", "hub+cliques", "grid64-w100", "er-selfloops")]
    code, mems, qs, sts = run_fused(eng, gs, gvl.GVL_MODE_DET, refine_random=1, seed=99)
    assert code == 0 and all(x == 0 for x in sts)
    for g, mem, q in zip(gs, mems, qs):
        o = oracle.leiden(g, mode=oracle.DET_SYNC, refine_random=1, seed=99)
        assert np.array_equal(mem, o.membership) and q == o.q, g.name


@pytest.mark.parametrize("name", ["rmat-s14", "planted-C1", "grid200-w100"])
def test_random_refinement_fast_quality(eng, name):
    g = graph(name)
    mem, q, _ = run(eng, g, gvl.GVL_MODE_FAST, refine_random=1, seed=7)
    assert q == oracle.modularity(g, mem)
    assert check(eng, g, mem)[0] == 0
    # the sequential oracle with the same randomized refinement and seed, on
    # the graph as numbered, minus 1e-3
    ref = oracle.leiden(g, mode=oracle.SEQ_ASYNC, refine_random=1, seed=7).q
    print("  random refinement %s: fast Q %.6f, sequential oracle %.6f, margin %+.6f" % (name, q, ref, q - ref),
          flush=True)
    assert q >= ref - 1e-3, (q, ref)


def test_option_values_checked(eng):
    g = graph("ring10xK5")
    for kw in ({"louvain": 2}, {"refine_random": -1}):
        with pytest.raises(gvl.GvlError):
            run(eng, g, gvl.GVL_MODE_FAST, **kw)


# ------------------------------------------------------------ gather probe ---

def test_gather_probe_sums_the_gathered_entries(eng):
    # the measurement aid bench.py times: sum of table[idx[e]]
    g = graph("rmat-s12")
    idx = torch.from_numpy(g.indices.astype(np.int32)).cuda()
    table = torch.randint(0, 1000, (g.n,), dtype=torch.int32, device="cuda",
                          generator=torch.Generator(device="cuda").manual_seed(5))
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    gvl.gvl_gather_probe(eng.ctx, idx.data_ptr(), idx.numel(), table.data_ptr(), g.n, sink.data_ptr())
    torch.cuda.synchronize()
    assert int(sink.item()) == int(table.long()[idx.long()].sum().item())
    bad = torch.tensor([g.n, -1, 5], dtype=torch.int32, device="cuda")  # outside the table: entry 0
    sink.zero_()
    gvl.gvl_gather_probe(eng.ctx, bad.data_ptr(), 3, table.data_ptr(), g.n, sink.data_ptr())
    torch.cuda.synchronize()
    assert int(sink.item()) == 2 * int(table[0].item()) + int(table[5].item())
    with pytest.raises(gvl.GvlError):
        gvl.gvl_gather_probe(eng.ctx, idx.data_ptr(), -1, table.data_ptr(), g.n, sink.data_ptr())
