"""Writes the full-size oracle records that the GPU's deterministic mode
must reproduce bit for bit, and that the fast mode's quality is held to:

  rmat_s24_oracle.json    R-MAT scale 24, edge factor 16 (the benchmark graph)
  grid4096_oracle.json    4096 x 4096 grid, 10 % of lattice edges dropped,
                          1 % diagonal shortcuts, integer weights 1..100
                          (total weight above 2^31: the gain keys of the
                          deterministic mode need more than 64 bits)

Each record holds the sequential oracle's modularity (the fast mode's
quality reference), and the deterministic oracle's modularity, pass count,
community count and a SHA-256 of its membership (int32, little endian).
The R-MAT record also holds the sequential oracle with the low-shrink
variant that leaves vertices without arcs out of the ratio.  Calls only the
seeded generators and the oracle; R-MAT takes ~20 minutes and ~12 GB of RAM,
the grid a few minutes.

    python tests/golden/make_fullsize_reference.py rmat_s24
    python tests/golden/make_fullsize_reference.py grid4096
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

import gen  # noqa: E402
import oracle  # noqa: E402

CONFIGS = {
    "rmat_s24": ("R-MAT scale 24, edge factor 16, a=.57 b=.19 c=.19, seed 2 (gen.rmat)",
                 lambda: gen.rmat(24, 16, 0.57, 0.19, 0.19, seed=2), True),
    "grid4096": ("grid 4096 x 4096, drop 0.1, diagonals 0.01, weights U{1..100}, seed 3 (gen.grid)",
                 lambda: gen.grid(4096, 4096, seed=3), False),
}


def record(name):
    title, make, variant = CONFIGS[name]
    t0 = time.time()
    g = make()
    t1 = time.time()
    r = oracle.leiden(g, mode=oracle.SEQ_ASYNC)
    t2 = time.time()
    d = oracle.leiden(g, mode=oracle.DET_SYNC)
    t3 = time.time()
    w = g.weights.astype("float64")
    out = {"graph": title, "vertices": g.n, "arcs": g.m, "total_weight": float(w.sum()),
           "mode": "sequential oracle (oracle.SEQ_ASYNC)",
           "modularity": r.q, "passes": len(r.passes), "termination": r.termination,
           "communities": int(r.membership.max()) + 1, "oracle_seconds": round(t2 - t1, 1),
           "generation_seconds": round(t1 - t0, 1),
           "det": {"mode": "deterministic oracle (oracle.DET_SYNC, default options)", "modularity": d.q,
                   "passes": len(d.passes), "termination": d.termination,
                   "communities": int(d.membership.max()) + 1,
                   "membership_sha256": hashlib.sha256(d.membership.astype("<i4").tobytes()).hexdigest(),
                   "oracle_seconds": round(t3 - t2, 1)}}
    del d
    if variant:
        t4 = time.time()
        v = oracle.leiden(g, mode=oracle.SEQ_ASYNC, shrink_excludes_isolated=1)
        out["shrink_excludes_isolated"] = {
            "mode": "sequential oracle, low-shrink ratio without vertices that have no arcs",
            "modularity": v.q, "passes": len(v.passes), "termination": v.termination,
            "communities": int(v.membership.max()) + 1, "oracle_seconds": round(time.time() - t4, 1)}
    with open(os.path.join(HERE, name + "_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    for name in sys.argv[1:] or list(CONFIGS):
        record(name)
