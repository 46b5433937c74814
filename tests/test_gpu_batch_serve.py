"""GPU tests of batched and served Leiden (many independent graphs on one GPU).

Every graph of a batch, and every request of a served mix, must get the
result it gets alone: bit-identical membership and modularity in
deterministic mode (and identical to the oracle's det-sync run), the fast
mode's quality bar in fast mode.  The server must respect its HBM arena,
admit requests as memory frees up, overlap requests on the device, reject a
request that can never fit and cancel one that still waits.
"""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2312_13936_amd as gvl  # noqa: E402
from test_gpu_parity import ASYNC_TRIES, WIDER_BAR as _SOLO_WIDER, async_bar, check_fast_run  # noqa: E402

FAST_TOL = 1e-3
# Per-graph margins wider than 1e-3 (by generated graph name), by the rules
# (i) and (ii) stated in test_gpu_parity.py:
#   lfr-14820-7017   (i) sequential spread 5.3e-3 over numberings (0.6583 ..
#                    0.6636); asynchronous lane-pool runs -4.7e-3 .. +0.7e-3
#   lfr-24108-14000  (ii) det oracle -0.97e-3 (sequential spread 1.8e-4)
#   lfr-13658-14004  (ii) det oracle -0.96e-3 (spread 2.7e-4)
#   lfr-14903-12006  (ii) det oracle -0.73e-3 (spread 1.5e-4); asynchronous
#                    serving runs -0.8e-3
WIDER_BAR = {"rmat-s12-ef16": _SOLO_WIDER["rmat-s12"], "er-300-0.03-9": _SOLO_WIDER["er-selfloops"],
             "grid-64x64": _SOLO_WIDER["grid64-w100"], "lfr-14820-7017": 5.5e-3, "lfr-24108-14000": 1.5e-3,
             "lfr-13658-14004": 1.5e-3, "lfr-14903-12006": 1.5e-3}


def lfr_mix(count, lo, hi, seed, mu=0.3, avg_deg=12.0):
    sizes = gen.lfr_sizes(count, lo, hi, seed)
    return [gen.lfr(int(n), avg_deg=avg_deg, mu=mu, seed=seed * 1000 + k) for k, n in enumerate(sizes)]


def dev(g):
    d = torch.device("cuda", 0)
    off = torch.from_numpy(g.offsets.astype(np.int32)).to(d)
    idx = torch.from_numpy(g.indices.astype(np.int32)).to(d)
    w = torch.from_numpy(g.weights.astype(np.float32)).to(d)
    return off, idx, w


@pytest.fixture(scope="module")
def eng():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    e = gvl.Leiden(0)
    yield e
    e.close()


def solo(eng, g, mode):
    off, idx, w = dev(g)
    r = eng.run(off, idx, w, 1.0, eng.options(mode))
    torch.cuda.synchronize()
    return r.membership.cpu().numpy(), r.modularity


def batch_graphs():
    gs = lfr_mix(18, 1000, 30000, seed=7)
    gs += [gen.ring_of_cliques(10, 5), gen.from_edges(2000, [(0, i) for i in range(1, 2000)]),
           gen.from_edges(500, [(i, i + 1) for i in range(499)]), gen.rmat(12, 16, seed=2),
           gen.from_edges(7, [])]
    return gs


def run_batch(eng, gs, mode, lanes, corrupt=None, **kw):
    tensors = [dev(g) for g in gs]
    mems = [torch.full((max(g.n, 1),), -7, dtype=torch.int32, device="cuda") for g in gs]
    if corrupt is not None:  # a decreasing offset makes that graph's CSR invalid
        tensors[corrupt][0][1] = tensors[corrupt][0][-1] + 1
    descs = [gvl.graph_desc(o, i, w, mm) for (o, i, w), mm in zip(tensors, mems)]
    opt = eng.options(mode, **kw)
    wsb = gvl.gvl_batch_workspace_bytes(descs, opt, lanes)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    code, qs, sts = gvl.gvl_leiden_batch(eng.ctx, descs, opt, lanes, ws.data_ptr(), wsb)
    torch.cuda.synchronize()
    return code, [m[:g.n].cpu().numpy() for m, g in zip(mems, gs)], qs, sts


@pytest.mark.parametrize("lanes", [1, 4, 8])
def test_batch_det_matches_solo_and_oracle(eng, lanes):
    gs = batch_graphs()
    print("batch det: %d graphs, %d lanes" % (len(gs), lanes), flush=True)
    code, mems, qs, sts = run_batch(eng, gs, gvl.GVL_MODE_DET, lanes)
    assert code == 0 and all(s == 0 for s in sts)
    for g, mem, q in zip(gs, mems, qs):
        m1, q1 = solo(eng, g, gvl.GVL_MODE_DET)
        assert np.array_equal(mem, m1), g.name
        assert q == q1, g.name
        if lanes == 4:
            o = oracle.leiden(g, mode=oracle.DET_SYNC)
            assert np.array_equal(mem, o.membership), g.name
            assert q == o.q, g.name


def check_fast_mix(gs, mems, qs):
    """Fast-mode bar over a mix, graph by graph: every result reports Eq. 1
    of its membership, has no disconnected community and reaches the
    sequential oracle's modularity on the graph as numbered minus 1e-3 (or
    the wider margin that WIDER_BAR states for that graph)."""
    short = []
    for g, mem, q in zip(gs, mems, qs):
        check_fast_run(g, mem, q)
        if g.m == 0:
            continue
        q0 = oracle.leiden(g, mode=oracle.SEQ_ASYNC).q
        tol = WIDER_BAR.get(g.name, FAST_TOL)
        print("  %s: fast Q %.6f, sequential oracle %.6f, margin %+.6f" % (g.name, q, q0, q - q0), flush=True)
        if q < q0 - tol:
            short.append("%s: fast Q %.6f vs sequential oracle %.6f" % (g.name, q, q0))
    assert not short, "; ".join(short)


def check_async_mix(gs, once):
    """The asynchronous schedule's bar over a mix (the rule stated with
    ASYNC_TRIES in test_gpu_parity.py): once() runs the whole mix and returns
    (memberships, modularities); every run's results must report Eq. 1 and
    have no disconnected community, and for each graph the best of up to
    ASYNC_TRIES runs must reach its bar."""
    bars = {k: async_bar(g, g.name, WIDER_BAR.get(g.name, FAST_TOL)) for k, g in enumerate(gs) if g.m > 0}
    best = {k: -np.inf for k in bars}
    for t in range(ASYNC_TRIES):
        mems, qs = once()
        for g, mem, q in zip(gs, mems, qs):
            check_fast_run(g, mem, q)
        for k, (q0, bar) in bars.items():
            best[k] = max(best[k], qs[k])
        short = [k for k, (q0, bar) in bars.items() if best[k] < bar]
        print("  try %d: %d of %d graphs below their bar" % (t, len(short), len(bars)), flush=True)
        if not short:
            return
    assert not short, "; ".join("%s: best fast Q %.6f vs sequential oracle %.6f (bar %.6f)" % (
        gs[k].name, best[k], bars[k][0], bars[k][1]) for k in short)


def test_batch_fast_quality(eng):
    gs = batch_graphs()
    print("batch fast: %d graphs" % len(gs), flush=True)

    def once():
        code, mems, qs, sts = run_batch(eng, gs, gvl.GVL_MODE_FAST, 6, sync_moves=0)
        assert code == 0
        return mems, qs
    check_async_mix(gs, once)


def test_batch_bad_graph_in_mix(eng):
    gs = batch_graphs()[:8]
    code, mems, qs, sts = run_batch(eng, gs, gvl.GVL_MODE_DET, 4, corrupt=3)
    assert code == -10  # GVL_E_BATCH
    assert sts[3] == -2 and all(s == 0 for k, s in enumerate(sts) if k != 3)
    for k, g in enumerate(gs):
        if k != 3:
            assert np.array_equal(mems[k], solo(eng, g, gvl.GVL_MODE_DET)[0]), g.name


def test_batch_workspace_checks(eng):
    gs = batch_graphs()[:3]
    tensors = [dev(g) for g in gs]
    mems = [torch.empty(g.n, dtype=torch.int32, device="cuda") for g in gs]
    descs = [gvl.graph_desc(o, i, w, mm) for (o, i, w), mm in zip(tensors, mems)]
    opt = eng.options(gvl.GVL_MODE_DET)
    wsb = gvl.gvl_batch_workspace_bytes(descs, opt, 2)
    assert wsb == 2 * max(-(-gvl.gvl_workspace_bytes(g.n, g.m, opt) // 256) * 256 for g in gs)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    with pytest.raises(gvl.GvlError) as e:
        gvl.gvl_leiden_batch(eng.ctx, descs, opt, 2, ws.data_ptr(), wsb - 1)
    assert e.value.code == -6
    code, qs, sts = gvl.gvl_leiden_batch(eng.ctx, [], opt, 2, ws.data_ptr(), wsb)
    assert code == 0 and qs == []


# ------------------------------------------------------------- fused batch ---

def run_fused(eng, gs, mode, resolutions=None, corrupt=None, **kw):
    tensors = [dev(g) for g in gs]
    mems = [torch.full((max(g.n, 1),), -7, dtype=torch.int32, device="cuda") for g in gs]
    if corrupt is not None:
        tensors[corrupt][0][1] = tensors[corrupt][0][-1] + 1
    res = resolutions or [1.0] * len(gs)
    descs = [gvl.graph_desc(o, i, w, mm, r) for (o, i, w), mm, r in zip(tensors, mems, res)]
    opt = eng.options(mode, **kw)
    wsb = gvl.gvl_fused_workspace_bytes(descs, opt)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    code, qs, sts = gvl.gvl_leiden_fused(eng.ctx, descs, opt, ws.data_ptr(), wsb)
    torch.cuda.synchronize()
    return code, [m[:g.n].cpu().numpy() for m, g in zip(mems, gs)], qs, sts


def solo_opts(eng, g, mode, resolution=1.0, **kw):
    off, idx, w = dev(g)
    r = eng.run(off, idx, w, resolution, eng.options(mode, **kw))
    torch.cuda.synchronize()
    return r.membership.cpu().numpy(), r.modularity


def fused_graphs():
    from test_gpu_parity import GRAPHS
    gs = batch_graphs()
    gs += [GRAPHS[k]() for k in ("hubs-wide", "hub+cliques", "grid64-w100", "er-selfloops", "planted-small")]
    return gs


def test_fused_det_matches_solo(eng):
    gs = fused_graphs()
    print("fused det: %d graphs" % len(gs), flush=True)
    code, mems, qs, sts = run_fused(eng, gs, gvl.GVL_MODE_DET)
    assert code == 0 and all(x == 0 for x in sts), sts
    for g, mem, q in zip(gs, mems, qs):
        m1, q1 = solo(eng, g, gvl.GVL_MODE_DET)
        assert np.array_equal(mem, m1), g.name
        assert q == q1, g.name


def test_fused_det_resolutions_and_subsweeps(eng):
    gs = lfr_mix(8, 1000, 20000, seed=17) + [gen.ring_of_cliques(30, 3), gen.rmat(12, 16, seed=2)]
    res = [0.5, 1.0, 1.5, 0.25, 2.0, 1.0, 0.75, 1.25, 1.0, 0.5]
    code, mems, qs, sts = run_fused(eng, gs, gvl.GVL_MODE_DET, resolutions=res, subsweeps=7)
    assert code == 0
    for g, r, mem, q in zip(gs, res, mems, qs):
        m1, q1 = solo_opts(eng, g, gvl.GVL_MODE_DET, r, subsweeps=7)
        assert np.array_equal(mem, m1), (g.name, r)
        assert q == q1, (g.name, r)
        o = oracle.leiden(g, mode=oracle.DET_SYNC, resolution=r, subsweeps=7)
        assert np.array_equal(mem, o.membership) and q == o.q, (g.name, r)


@pytest.mark.parametrize("sync_moves", [3, 0])
def test_fused_fast_quality(eng, sync_moves):
    gs = fused_graphs()

    def once():
        code, mems, qs, sts = run_fused(eng, gs, gvl.GVL_MODE_FAST, sync_moves=sync_moves)
        assert code == 0
        return mems, qs
    if sync_moves == 3:
        check_fast_mix(gs, *once())
    else:
        check_async_mix(gs, once)


def test_fused_fast_sync_matches_solo(eng):
    gs = batch_graphs()
    code, mems, qs, sts = run_fused(eng, gs, gvl.GVL_MODE_FAST, sync_moves=3)
    assert code == 0
    for g, mem, q in zip(gs, mems, qs):
        m1, q1 = solo_opts(eng, g, gvl.GVL_MODE_FAST, sync_moves=3)
        assert np.array_equal(mem, m1), g.name
        assert q == q1, g.name


def test_fused_bad_graph_in_mix(eng):
    gs = batch_graphs()[:8]
    code, mems, qs, sts = run_fused(eng, gs, gvl.GVL_MODE_DET, corrupt=3)
    assert code == -10
    assert sts[3] == -2 and all(x == 0 for k, x in enumerate(sts) if k != 3)
    for k, g in enumerate(gs):
        if k != 3:
            assert np.array_equal(mems[k], solo(eng, g, gvl.GVL_MODE_DET)[0]), g.name


def test_fused_noninteger_weights_det(eng):
    g = gen.ring_of_cliques(10, 5)
    h = gen.Graph(g.n, g.m, g.offsets, g.indices, g.weights * 0.5, None, "half-weights")
    code, mems, qs, sts = run_fused(eng, [g, h, g], gvl.GVL_MODE_DET)
    assert code == -10 and sts == [0, -4, 0]
    assert np.array_equal(mems[0], mems[2]) and qs[0] == qs[2]


# ------------------------------------------------------------------ serving ---

WAIT_MS = 60000  # a request that is not done by then fails the test (GVL_E_BUSY)


def footprint(g, opt):
    return -(-gvl.gvl_workspace_bytes(g.n, g.m, opt) // 256) * 256


def serve(gs, tensors, mode, lanes, arena_bytes, alone, **kw):
    opt = gvl.Leiden.options(mode, **kw)
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    mems = [torch.full((max(g.n, 1),), -7, dtype=torch.int32, device="cuda") for g in gs]
    torch.cuda.synchronize()
    srv = gvl.Server(arena, lanes, opt)
    out = []
    try:
        if alone:
            for g, (o, i, w), mm in zip(gs, tensors, mems):
                t = srv.submit(o, i, w, mm)
                info = srv.wait(t, WAIT_MS)
                assert info.state == gvl.GVL_REQ_DONE and info.result == 0
                out.append((mm[:g.n].cpu().numpy(), info.modularity))
                srv.release(t)
        else:
            tickets = [srv.submit(o, i, w, mm) for (o, i, w), mm in zip(tensors, mems)]
            for g, t, mm in zip(gs, tickets, mems):
                info = srv.wait(t, WAIT_MS)
                assert info.state == gvl.GVL_REQ_DONE and info.result == 0
                assert info.latency_ms >= info.queue_ms >= 0
                out.append((mm[:g.n].cpu().numpy(), info.modularity))
                srv.release(t)
        st = srv.stats()
    finally:
        srv.close()
    return out, st


def test_serve_alone_vs_mix_det(eng):
    gs = lfr_mix(16, 2000, 60000, seed=11, avg_deg=16.0)
    tensors = [dev(g) for g in gs]
    opt = gvl.Leiden.options(gvl.GVL_MODE_DET)
    arena = 8 * max(footprint(g, opt) for g in gs)
    print("serve det: %d requests, arena %d MB" % (len(gs), arena >> 20), flush=True)
    alone, _ = serve(gs, tensors, gvl.GVL_MODE_DET, 4, arena, alone=True)
    mix, st = serve(gs, tensors, gvl.GVL_MODE_DET, 4, arena, alone=False)
    for g, (m1, q1), (m2, q2) in zip(gs, alone, mix):
        assert np.array_equal(m1, m2), g.name
        assert q1 == q2, g.name
    for g, (m, q) in zip(gs[:6], mix[:6]):
        o = oracle.leiden(g, mode=oracle.DET_SYNC)
        assert np.array_equal(m, o.membership) and q == o.q, g.name
    assert st.completed == len(gs) and st.pending == 0 and st.running == 0
    assert st.max_running >= 2  # requests overlapped on the device
    assert st.arena_peak <= st.arena_bytes and st.arena_used == 0


def test_serve_mix_fast_quality(eng):
    gs = lfr_mix(10, 2000, 40000, seed=12, avg_deg=16.0)
    tensors = [dev(g) for g in gs]
    opt = gvl.Leiden.options(gvl.GVL_MODE_FAST)
    arena = 6 * max(footprint(g, opt) for g in gs)
    print("serve fast: %d requests" % len(gs), flush=True)

    # asynchronous commits make every run differ a little, alone or in a
    # mix, so the mix is held to the asynchronous schedule's quality bar
    def once():
        mix, st = serve(gs, tensors, gvl.GVL_MODE_FAST, 4, arena, alone=False, sync_moves=0)
        return [m for m, _ in mix], [q for _, q in mix]
    check_async_mix(gs, once)


def test_serve_alone_vs_mix_fast_sync(eng):
    # fast mode (FP64 gains) with group-synchronous moves is reproducible, so
    # a served result must be identical alone and in a mix
    gs = lfr_mix(10, 2000, 40000, seed=14, avg_deg=16.0)
    tensors = [dev(g) for g in gs]
    opt = gvl.Leiden.options(gvl.GVL_MODE_FAST, sync_moves=3)
    arena = 6 * max(footprint(g, opt) for g in gs)
    alone, _ = serve(gs, tensors, gvl.GVL_MODE_FAST, 4, arena, alone=True, sync_moves=3)
    mix, st = serve(gs, tensors, gvl.GVL_MODE_FAST, 4, arena, alone=False, sync_moves=3)
    for g, (m1, q1), (m2, q2) in zip(gs, alone, mix):
        assert np.array_equal(m1, m2), g.name
        assert q1 == q2, g.name
    assert st.max_running >= 2
    check_fast_mix(gs, [m for m, _ in mix], [q for _, q in mix])


def test_serve_admission_by_footprint(eng):
    # an arena that holds two of these workspaces at a time: the rest wait
    # and are admitted as earlier requests finish
    gs = [gen.lfr(25000, seed=13000 + k) for k in range(8)]  # nearly equal footprints
    tensors = [dev(g) for g in gs]
    opt = gvl.Leiden.options(gvl.GVL_MODE_DET)
    fp = max(footprint(g, opt) for g in gs)
    print("serve admission: arena %.1f workspaces" % 2.5, flush=True)
    assert 3 * min(footprint(g, opt) for g in gs) > 2 * fp + fp // 2
    mix, st = serve(gs, tensors, gvl.GVL_MODE_DET, 4, 2 * fp + fp // 2, alone=False)
    assert st.max_running <= 2
    assert st.arena_peak <= st.arena_bytes
    for g, (m, q) in zip(gs, mix):
        m1, q1 = solo(eng, g, gvl.GVL_MODE_DET)
        assert np.array_equal(m, m1) and q == q1, g.name


def test_serve_errors_and_cancel(eng):
    big = gen.lfr(60000, seed=21)
    small = gen.lfr(3000, seed=22)
    tb, ts = dev(big), dev(small)
    mb = torch.empty(big.n, dtype=torch.int32, device="cuda")
    ms = [torch.empty(small.n, dtype=torch.int32, device="cuda") for _ in range(2)]
    opt = gvl.Leiden.options(gvl.GVL_MODE_DET)
    arena = torch.empty(footprint(big, opt) + 4096, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    print("serve errors and cancel", flush=True)
    srv = gvl.Server(arena, 1, opt)
    try:
        # a request whose workspace can never fit is refused at submission
        huge = gvl.gvl_graph_desc(big.n * 4, big.m * 4, tb[0].data_ptr(), tb[1].data_ptr(), tb[2].data_ptr(), 1.0,
                                  mb.data_ptr())
        with pytest.raises(gvl.GvlError) as e:
            gvl.gvl_server_submit(srv.srv, huge)
        assert e.value.code == -6
        nomem = gvl.gvl_graph_desc(small.n, small.m, ts[0].data_ptr(), ts[1].data_ptr(), None, 1.0, None)
        with pytest.raises(gvl.GvlError) as e:
            gvl.gvl_server_submit(srv.srv, nomem)
        assert e.value.code == -1
        t1 = srv.submit(*tb, mb)
        t2 = srv.submit(*ts, ms[0])
        t3 = srv.submit(*ts, ms[1])
        # one lane: t3 still waits unless t1 and t2 have both finished already
        try:
            srv.cancel(t3)
            cancelled = True
        except gvl.GvlError as e:
            assert e.code == -9
            cancelled = False
        i1, i2, i3 = srv.wait(t1, WAIT_MS), srv.wait(t2, WAIT_MS), srv.wait(t3, WAIT_MS)
        assert i1.state == gvl.GVL_REQ_DONE and i2.state == gvl.GVL_REQ_DONE
        assert i3.state == (gvl.GVL_REQ_CANCELLED if cancelled else gvl.GVL_REQ_DONE)
        with pytest.raises(gvl.GvlError) as e:
            srv.cancel(t1)  # already done
        assert e.value.code == -9
        assert np.array_equal(mb.cpu().numpy(), solo(eng, big, gvl.GVL_MODE_DET)[0])
        assert np.array_equal(ms[0].cpu().numpy(), solo(eng, small, gvl.GVL_MODE_DET)[0])
        for t in (t1, t2, t3):
            srv.release(t)
        with pytest.raises(gvl.GvlError) as e:
            srv.poll(t1)  # released
        assert e.value.code == -1
        assert srv.stats().arena_used == 0
    finally:
        srv.close()
