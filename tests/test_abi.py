"""CPU-side checks of the C-ABI library: it loads, exports every symbol that
include/gvl.h declares, and its host-only entry points behave (no GPU work)."""
import os
import re

import pytest

import paper_2312_13936_amd as gvl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gvl.h")).read()
    return sorted(set(re.findall(r"\b(gvl_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gvl.LIB_PATH):
        from paper_2312_13936_amd import build
        build.build()
    return gvl.load_library()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert {"gvl_create", "gvl_leiden", "gvl_workspace_bytes", "gvl_modularity"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(gvl.EXPORTS) == names


def test_default_options(lib):
    fast = gvl.gvl_default_options(gvl.GVL_MODE_FAST)
    det = gvl.gvl_default_options(gvl.GVL_MODE_DET)
    # Sec. 4.1 constants
    for o in (fast, det):
        assert o.tolerance == 0.01 and o.tolerance_drop == 10.0
        assert o.aggregation_tolerance == 0.8 and o.max_iterations == 20 and o.max_passes == 20
    # sub-sweep groups: deterministic 32 (the oracle's default); fast 0 = by the longest row
    assert fast.mode == 0 and det.mode == 1 and det.subsweeps == 32 and fast.subsweeps == 0
    assert fast.sync_moves == 3 and fast.refine_sweeps == 20 and fast.max_passes == 20
    with pytest.raises(gvl.GvlError):
        gvl.gvl_default_options(7)


def test_workspace_bytes_grows_with_size(lib):
    o = gvl.gvl_default_options(gvl.GVL_MODE_FAST)
    d = gvl.gvl_default_options(gvl.GVL_MODE_DET)
    a = gvl.gvl_workspace_bytes(1000, 10000, o)
    b = gvl.gvl_workspace_bytes(2000, 10000, o)
    c = gvl.gvl_workspace_bytes(1000, 20000, o)
    assert 0 < a < b and a < c
    assert gvl.gvl_workspace_bytes(1000, 20000, d) > c  # det stores super-graph weights as float64
    assert gvl.gvl_workspace_bytes(0, 0, o) > 0
    with pytest.raises(gvl.GvlError):
        gvl.gvl_workspace_bytes(-1, 0, o)


def test_status_strings(lib):
    assert gvl.gvl_status_string(0) == "ok"
    assert "workspace" in gvl.gvl_status_string(-6)
    assert gvl.gvl_status_string(12345) == "unknown status"


def test_tuning_table_validation_and_classes(lib):
    assert gvl.gvl_graph_class(10000, 147000) == gvl.GVL_CLASS_SMALL
    assert gvl.gvl_graph_class(16777216, 61047992) == gvl.GVL_CLASS_LOWDEG
    assert gvl.gvl_graph_class(16777216, 520764976) == gvl.GVL_CLASS_SKEWED
    assert gvl.gvl_graph_class(100, 10, fused=True) == gvl.GVL_CLASS_BATCH
    saved = [gvl.gvl_get_tuning(c) for c in range(gvl.GVL_NUM_CLASSES)]
    try:
        t = gvl.gvl_tuning.from_buffer_copy(saved[0])
        t.bin_max[4] = 64
        t.decide_grid = 512
        gvl.gvl_set_tuning(gvl.GVL_CLASS_SMALL, t)
        got = gvl.gvl_get_tuning(gvl.GVL_CLASS_SMALL)
        assert list(got.bin_max)[4] == 64 and got.decide_grid == 512
        for bad in (dict(b=4, v=256), dict(b=5, v=128), dict(b=3, v=8)):  # above compiled, below 256, decreasing
            u = gvl.gvl_tuning.from_buffer_copy(saved[0])
            u.bin_max[bad["b"]] = bad["v"]
            with pytest.raises(gvl.GvlError):
                gvl.gvl_set_tuning(gvl.GVL_CLASS_SMALL, u)
        u = gvl.gvl_tuning.from_buffer_copy(saved[0])
        u.agg_grid = 0
        with pytest.raises(gvl.GvlError):
            gvl.gvl_set_tuning(gvl.GVL_CLASS_SMALL, u)
        with pytest.raises(gvl.GvlError):
            gvl.gvl_set_tuning(7, saved[0])
    finally:
        for c, t in enumerate(saved):
            gvl.gvl_set_tuning(c, t)


def test_tuning_file_is_parsed(lib, tmp_path, capfd):
    saved = [gvl.gvl_get_tuning(c) for c in range(gvl.GVL_NUM_CLASSES)]
    p = tmp_path / "tune.txt"
    p.write_text("# comment\nlowdeg 4 8 16 16 64 512 2048 1024 8192  # trailing comment\n"
                 "skewed 4 8 16 32 256 1024 1024 2048 4096\nunknown 1 2 3\n")
    try:
        gvl.gvl_load_tuning(str(p))
        t = gvl.gvl_get_tuning(gvl.GVL_CLASS_LOWDEG)
        assert list(t.bin_max) == [4, 8, 16, 16, 64, 512] and (t.decide_grid, t.commit_grid, t.agg_grid) == (2048, 1024,
                                                                                                          8192)
        # the invalid lines (bin 4 above 128; unknown class) are skipped and reported
        assert list(gvl.gvl_get_tuning(gvl.GVL_CLASS_SKEWED).bin_max) == list(saved[gvl.GVL_CLASS_SKEWED].bin_max)
        err = capfd.readouterr().err
        assert "tune.txt:3" in err and "tune.txt:4" in err
        with pytest.raises(gvl.GvlError):
            gvl.gvl_load_tuning(str(tmp_path / "missing.txt"))
    finally:
        for c, t in enumerate(saved):
            gvl.gvl_set_tuning(c, t)
