#!/usr/bin/env python3
"""Benchmark of the Leiden hot path on one MI355X.

One step = one gvl_leiden call on a graph already resident in HBM: every
pass of local-moving, refinement and aggregation, the final relabelling and
the modularity, i.e. the whole hot path.  value = arcs of the symmetric CSR
(both directions, the paper's |E| convention) / seconds per step.

Default workload: R-MAT scale 24, edge factor 16, (a, b, c) = (.57, .19, .19),
symmetrised, self-loops and duplicates removed, unit weights stored FP32,
int32 CSR (seeded synthetic input).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Leiden edges/s at matched modularity; batched graphs/s vs plain; p99 latency"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "rmat-s24": dict(kind="rmat", scale=24, edge_factor=16, a=0.57, b=0.19, c=0.19, seed=2,
                     desc="R-MAT scale 24 (16.8M vertices), edge factor 16, a=.57 b=.19 c=.19, "
                          "symmetrised, no self-loops/duplicates, unit weights FP32, int32 CSR"),
    "planted-10k": dict(kind="planted", blocks=20, block_size=500, p_in=0.02, p_out=0.0005, seed=1,
                        desc="planted partition 20x500, p_in 0.02, p_out 0.0005, unit weights FP32"),
    "grid-4096": dict(kind="grid", rows=4096, cols=4096, drop=0.1, diag_frac=0.01, wmax=100, seed=3,
                      desc="4096x4096 grid, 10% edges dropped, 1% diagonal shortcuts, weights U{1..100}"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_graph(w):
    import gen
    if w["kind"] == "rmat":
        return gen.rmat(w["scale"], w["edge_factor"], w["a"], w["b"], w["c"], seed=w["seed"])
    if w["kind"] == "planted":
        return gen.planted(w["blocks"], w["block_size"], w["p_in"], w["p_out"], seed=w["seed"])
    if w["kind"] == "grid":
        return gen.grid(w["rows"], w["cols"], w["drop"], w["diag_frac"], w["wmax"], seed=w["seed"])
    raise KeyError(w["kind"])


def scan_bytes(st) -> float:
    """Algorithmic bytes of the neighbour-community scan kernels (local-moving
    and refinement decisions), from the work the kernels counted:
    per arc 12 B (neighbour id, weight, community of the neighbour), +4 B per
    refinement arc (bound label), per distinct candidate community 8 B
    (its total weight), per scanned vertex 29 B (two offsets, K, own label,
    own community total, flag), per move 20 B (label store, two totals)."""
    return (12.0 * st.scan_arcs + 4.0 * st.scan_refine_arcs + 8.0 * st.scan_candidates
            + 29.0 * st.scan_vertices + 20.0 * st.scan_moves)


def agg_bytes(st) -> float:
    """Algorithmic bytes of the aggregation row kernels: per arc read 12 B
    (neighbour id, weight, its super-vertex label), per arc written 8 B, per
    member vertex 12 B (member id, row offset, row length)."""
    return 12.0 * st.agg_arcs + 8.0 * st.agg_out_arcs + 12.0 * st.agg_vertices


def cpu_baseline(scale: int):
    """The oracle (sequential, one thread) on a bounded sample: R-MAT with the
    same parameters at a smaller scale."""
    import gen
    import oracle
    g = gen.rmat(scale, 16, 0.57, 0.19, 0.19, seed=2)
    t0 = time.perf_counter()
    r = oracle.leiden(g, mode=oracle.SEQ_ASYNC)
    dt = time.perf_counter() - t0
    return {"value": g.m / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": "sequential oracle on R-MAT scale %d (same a,b,c, edge factor 16): %d vertices, %d arcs, "
                      "%.1f s, Q=%.4f; CPU %s" % (scale, g.n, g.m, dt, r.q, platform.processor() or platform.machine()),
            "seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat-s24", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="fast", choices=["fast", "det"])
    ap.add_argument("--subsweeps", type=int, default=0, help="0 = library default")
    ap.add_argument("--cpu-sample-scale", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(graphs would shard by vertex ranges; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2312_13936_amd as gvl

    w = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    g = make_graph(w)
    log("generated %s: n=%d m=%d in %.1fs" % (args.workload, g.n, g.m, time.perf_counter() - t0))
    dev = torch.device("cuda", 0)
    off = torch.from_numpy(g.offsets).to(dev)
    idx = torch.from_numpy(g.indices).to(dev)
    wt = torch.from_numpy(g.weights).to(dev)
    torch.cuda.synchronize()

    eng = gvl.Leiden(0)
    mode = gvl.GVL_MODE_DET if args.mode == "det" else gvl.GVL_MODE_FAST
    kw = dict(profile=1)
    if args.subsweeps:
        kw["subsweeps"] = args.subsweeps
    opt = eng.options(mode, **kw)
    for k in range(args.warmup):
        r = eng.run(off, idx, wt, 1.0, opt)
        torch.cuda.synchronize()
        log("warmup %d: Q=%.6f passes=%d" % (k, r.modularity, r.stats.passes))
    times, qs, stats = [], [], []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for k in range(args.steps):
        t1 = time.perf_counter()
        r = eng.run(off, idx, wt, 1.0, opt)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        qs.append(r.modularity)
        stats.append(r.stats)
        log("step %d: %.1f ms Q=%.6f communities=%d passes=%d" % (k, 1e3 * times[-1], r.modularity,
                                                                  r.stats.num_communities, r.stats.passes))
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    ms_per_step = 1e3 * total / args.steps
    value = g.m / (total / args.steps)

    # roofline of the dominant kernel class (neighbour-community scan)
    sb = sum(scan_bytes(s) for s in stats)
    sms = sum(s.ms_scan_kernels for s in stats)
    ab = sum(agg_bytes(s) for s in stats)
    ams = sum(s.ms_agg_kernels for s in stats)
    scan_gbs = sb / (sms * 1e-3) / 1e9 if sms > 0 else 0.0
    agg_gbs = ab / (ams * 1e-3) / 1e9 if ams > 0 else 0.0
    last = stats[-1]
    phase = {"move_ms": last.ms_move, "refine_ms": last.ms_refine, "aggregate_ms": last.ms_aggregate,
             "other_ms": last.ms_other, "scan_kernels_ms": last.ms_scan_kernels,
             "agg_kernels_ms": last.ms_agg_kernels, "scan_launches": last.scan_launches,
             "agg_launches": last.agg_launches}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w["desc"], "vertices": g.n, "arcs": g.m, "mode": args.mode,
                   "subsweeps": opt.subsweeps, "resolution": 1.0, "tolerance": opt.tolerance,
                   "max_passes": opt.max_passes, "parallelism": "single GPU"},
        "modularity": float(np.median(qs)),
        "modularity_min": float(min(qs)),
        "communities": int(last.num_communities),
        "passes": int(last.passes),
        "phases": phase,
        "roofline": {"bound": "hbm", "kernel": "neighbour-community scan (k_decide_*: local-moving + refinement)",
                     "achieved": scan_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": scan_gbs / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_step": sb / len(stats),
                     "kernel_ms_per_step": sms / len(stats)},
        "roofline_aggregation": {"bound": "hbm", "kernel": "super-vertex rows (k_agg_*)", "achieved": agg_gbs,
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": agg_gbs / HBM_PEAK_GBS,
                                 "algorithmic_bytes_per_step": ab / len(stats),
                                 "kernel_ms_per_step": ams / len(stats)},
        "cpu_baseline": None,
    }
    eng.close()
    del off, idx, wt
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on R-MAT scale %d" % args.cpu_sample_scale)
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_scale)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
