"""Deterministic parity at the benchmark's full size.

The oracle's det-sync run on the R-MAT scale-24 graph (16.8M vertices,
521M arcs) is recorded in tests/golden/rmat_s24_oracle.json by
tests/golden/make_rmat_s24_reference.py (modularity and a SHA-256 of the
membership); the GPU's deterministic mode must reproduce both exactly, in
the launch configuration bench.py times.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2312_13936_amd as gvl  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rmat_s24_oracle.json")


def test_rmat_s24_det_bit_exact_at_full_size():
    rec = json.load(open(GOLDEN))
    g = gen.rmat(24, 16, 0.57, 0.19, 0.19, seed=2)
    assert (g.n, g.m) == (rec["vertices"], rec["arcs"])
    print("full-size det parity: R-MAT s24", g.n, g.m, flush=True)
    d = torch.device("cuda", 0)
    off = torch.from_numpy(g.offsets).to(d)
    idx = torch.from_numpy(g.indices).to(d)
    w = torch.from_numpy(g.weights).to(d)
    del g
    eng = gvl.Leiden(0)
    try:
        r = eng.run(off, idx, w, 1.0, eng.options(gvl.GVL_MODE_DET))
        torch.cuda.synchronize()
        mem = r.membership.cpu().numpy().astype("<i4")
    finally:
        eng.close()
    det = rec["det"]
    assert r.modularity == det["modularity"]
    assert int(mem.max()) + 1 == det["communities"]
    assert hashlib.sha256(mem.tobytes()).hexdigest() == det["membership_sha256"]
    assert r.stats.passes == det["passes"] and r.stats.termination == det["termination"]
