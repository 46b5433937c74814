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
    assert fast.mode == 0 and det.mode == 1 and det.subsweeps == 32 and fast.subsweeps == 32
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
