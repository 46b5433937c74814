"""gvl_leiden_static (the entry point for callers that cannot allocate device
memory) against gvl_leiden on the same inputs, through the C ABI: two calls
in a row, the second on a smaller graph (the shared device array keeps the
first call's contents), in deterministic mode (bit-identical results, also
equal to the oracle's) and in fast mode with group-synchronous moves
(reproducible, so also identical); oversized graphs and timing requests are
rejected."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2312_13936_amd as gvl  # noqa: E402


def dev(g):
    d = torch.device("cuda", 0)
    return (torch.from_numpy(g.offsets.astype(np.int32)).to(d), torch.from_numpy(g.indices.astype(np.int32)).to(d),
            torch.from_numpy(g.weights.astype(np.float32)).to(d))


def both(ctx, g, opt):
    off, idx, w = dev(g)
    d = torch.device("cuda", 0)
    m_ref = torch.full((g.n,), -3, dtype=torch.int32, device=d)
    m_sta = torch.full((g.n,), -5, dtype=torch.int32, device=d)
    wsb = gvl.gvl_workspace_bytes(g.n, g.m, opt)
    ws = torch.empty(wsb, dtype=torch.uint8, device=d)
    q_ref = gvl.gvl_leiden(ctx, g.n, g.m, off.data_ptr(), idx.data_ptr(), w.data_ptr(), 1.0, opt, ws.data_ptr(),
                           wsb, m_ref.data_ptr())
    torch.cuda.synchronize()
    st = gvl.gvl_stats()
    q_sta = gvl.gvl_leiden_static(ctx, g.n, g.m, off.data_ptr(), idx.data_ptr(), w.data_ptr(), 1.0, opt,
                                  m_sta.data_ptr(), st)
    torch.cuda.synchronize()
    return m_ref.cpu().numpy(), q_ref, m_sta.cpu().numpy(), q_sta, st


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    stream = torch.cuda.current_stream()
    c = gvl.gvl_create(0, stream.cuda_stream)
    yield c
    gvl.gvl_destroy(c)


@pytest.mark.parametrize("mode", [gvl.GVL_MODE_DET, gvl.GVL_MODE_FAST])
def test_static_matches_workspace_entry_point(ctx, mode):
    opt = gvl.gvl_default_options(mode)
    big = gen.lfr(150000, avg_deg=12.0, mu=0.3, seed=91)
    small = gen.planted(8, 120, 0.08, 0.004, seed=21)
    assert gvl.gvl_workspace_bytes(big.n, big.m, opt) <= gvl.GVL_STATIC_WORKSPACE_BYTES
    for g in (big, small):  # the second call finds the first call's contents in the array
        print("static vs workspace entry point:", g.name, g.n, g.m, "mode", mode, flush=True)
        m_ref, q_ref, m_sta, q_sta, st = both(ctx, g, opt)
        assert np.array_equal(m_ref, m_sta), g.name
        assert q_ref == q_sta, g.name
        assert st.passes >= 1
        if mode == gvl.GVL_MODE_DET:
            o = oracle.leiden(g, mode=oracle.DET_SYNC)
            assert np.array_equal(m_sta, o.membership) and q_sta == o.q


def test_static_rejects_oversize_and_profiling(ctx):
    opt = gvl.gvl_default_options(gvl.GVL_MODE_FAST)
    d = torch.device("cuda", 0)
    g = gen.planted(8, 120, 0.08, 0.004, seed=21)
    off, idx, w = dev(g)
    mem = torch.empty(g.n, dtype=torch.int32, device=d)
    # a graph whose workspace would exceed the array: checked before any device work
    n_big, m_big = 4_000_000, 64_000_000
    assert gvl.gvl_workspace_bytes(n_big, m_big, opt) > gvl.GVL_STATIC_WORKSPACE_BYTES
    with pytest.raises(gvl.GvlError) as e:
        gvl.gvl_leiden_static(ctx, n_big, m_big, off.data_ptr(), idx.data_ptr(), w.data_ptr(), 1.0, opt,
                              mem.data_ptr())
    assert e.value.code == -6
    prof = gvl.gvl_default_options(gvl.GVL_MODE_FAST)
    prof.profile = 1
    with pytest.raises(gvl.GvlError) as e:
        gvl.gvl_leiden_static(ctx, g.n, g.m, off.data_ptr(), idx.data_ptr(), w.data_ptr(), 1.0, prof,
                              mem.data_ptr())
    assert e.value.code == -1
    # still usable afterwards
    q = gvl.gvl_leiden_static(ctx, g.n, g.m, off.data_ptr(), idx.data_ptr(), w.data_ptr(), 1.0, opt, mem.data_ptr())
    assert q == oracle.modularity(g, mem.cpu().numpy())
