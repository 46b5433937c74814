"""Writes rmat_s24_oracle.json: the oracle on the R-MAT scale-24 benchmark
graph -- the sequential mode's modularity (the fast mode's quality
reference, reported by bench.py next to the GPU's), and the deterministic
mode's modularity and a SHA-256 of its membership (int32, little endian),
which the deterministic GPU path must reproduce bit for bit at full size.
Calls only the seeded generator and the oracle; takes ~15 minutes and
~12 GB of RAM.

    python tests/golden/make_rmat_s24_reference.py
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


def main():
    t0 = time.time()
    g = gen.rmat(24, 16, 0.57, 0.19, 0.19, seed=2)
    t1 = time.time()
    r = oracle.leiden(g, mode=oracle.SEQ_ASYNC)
    t2 = time.time()
    d = oracle.leiden(g, mode=oracle.DET_SYNC)
    t3 = time.time()
    out = {"graph": "R-MAT scale 24, edge factor 16, a=.57 b=.19 c=.19, seed 2 (gen.rmat)",
           "vertices": g.n, "arcs": g.m, "mode": "sequential oracle (oracle.SEQ_ASYNC)",
           "modularity": r.q, "passes": len(r.passes), "termination": r.termination,
           "communities": int(r.membership.max()) + 1, "oracle_seconds": round(t2 - t1, 1),
           "generation_seconds": round(t1 - t0, 1),
           "det": {"mode": "deterministic oracle (oracle.DET_SYNC, default options)", "modularity": d.q,
                   "passes": len(d.passes), "termination": d.termination,
                   "communities": int(d.membership.max()) + 1,
                   "membership_sha256": hashlib.sha256(d.membership.astype("<i4").tobytes()).hexdigest(),
                   "oracle_seconds": round(t3 - t2, 1)}}
    with open(os.path.join(HERE, "rmat_s24_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
