"""Autotuner of the launch shapes per class of graph; writes tune.txt next to
libgvl.so, which the library loads when its first context is created.

    python -m paper_2312_13936_amd.tune [--classes small,lowdeg,skewed,batch] [--reps 5] [--out PATH]

For each class it times gvl_leiden (fused batches: gvl_leiden_fused) on a
seeded synthetic graph of that class and does coordinate descent over the
tunable values: the largest row of the lane-group bins 2, 3, 4 (which lanes
per row a degree range gets), the largest row of the one-workgroup bin 5
(where rows move to the wide kernel), and the workgroups per decision,
commit and aggregation launch.  The first measurement is discarded (it
pays for first-touch and graph instantiation), and a value replaces the
current one only when it is faster by more than MIN_GAIN, above the
run-to-run noise of these workloads (about 1 %).  The values never change a result (the
deterministic mode is bit-identical under any of them; the GPU tests check
it), only which kernel handles a row and how many workgroups a launch has.
Needs a GPU.
"""
from __future__ import annotations

import argparse
import os
import statistics
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import paper_2312_13936_amd as gvl  # noqa: E402

# (tuning field, bin index or None, candidate values)
KNOBS = [("bin_max", 2, (8, 16)), ("bin_max", 3, (16, 32)), ("bin_max", 4, (32, 64, 128)),
         ("bin_max", 5, (256, 512, 1024)), ("decide_grid", None, (256, 512, 1024, 2048, 4096)),
         ("commit_grid", None, (512, 1024, 2048, 4096)), ("agg_grid", None, (1024, 2048, 4096, 8192))]
MIN_GAIN = 0.02

WORKLOADS = {
    "small": "planted partition 20 x 500 (p_in 0.02, p_out 0.0005) and an LFR-style graph of 100k vertices",
    "lowdeg": "4096 x 4096 grid, 10 % of edges dropped, 1 % diagonals, weights 1..100",
    "skewed": "R-MAT scale 24, edge factor 16, a=.57 b=.19 c=.19",
    "batch": "512 LFR-style graphs of 1k-200k vertices (the batched workload's recipe, first 512 graphs)",
}


def make(cls):
    import gen
    if cls == "small":
        return [gen.planted(20, 500, 0.02, 0.0005, seed=1), gen.lfr(100000, avg_deg=12.0, mu=0.3, seed=77)]
    if cls == "lowdeg":
        return [gen.grid(4096, 4096, seed=3)]
    if cls == "skewed":
        return [gen.rmat(24, 16, 0.57, 0.19, 0.19, seed=2)]
    sizes = gen.lfr_sizes(4096, 1000, 200000, 4096)[:512]
    return [gen.lfr(int(n), avg_deg=12.0, mu=0.3, seed=1000 + k) for k, n in enumerate(sizes)]


def timer(cls, graphs, reps):
    import torch
    d = torch.device("cuda", 0)
    tens = [(torch.from_numpy(g.offsets).to(d), torch.from_numpy(g.indices).to(d), torch.from_numpy(g.weights).to(d))
            for g in graphs]
    eng = gvl.Leiden(0)
    opt = eng.options(gvl.GVL_MODE_FAST)
    if cls == "batch":
        mems = [torch.empty(max(g.n, 1), dtype=torch.int32, device=d) for g in graphs]
        descs = [gvl.graph_desc(o, i, w, m) for (o, i, w), m in zip(tens, mems)]
        wsb = gvl.gvl_fused_workspace_bytes(descs, opt)
        ws = torch.empty(wsb, dtype=torch.uint8, device=d)

        def once():
            code, _, _ = gvl.gvl_leiden_fused(eng.ctx, descs, opt, ws.data_ptr(), wsb)
            assert code == 0
    else:
        def once():
            for t in tens:
                eng.run(*t, 1.0, opt)

    def measure():
        once()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            once()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return 1e3 * statistics.median(ts)
    return measure


def get(t, field, b):
    return getattr(t, field)[b] if b is not None else getattr(t, field)


def put(t, field, b, v):
    if b is not None:
        getattr(t, field)[b] = v
    else:
        setattr(t, field, v)


def tune(cls, reps, log):
    c = gvl.CLASS_NAMES.index(cls)
    graphs = make(cls)
    measure = timer(cls, graphs, reps)
    best = gvl.gvl_get_tuning(c)
    gvl.gvl_set_tuning(c, best)
    measure()  # discarded
    base = measure()
    cur = base
    notes = ["%s: %s; default %.2f ms" % (cls, WORKLOADS[cls], base)]
    log(notes[0])
    for field, b, values in KNOBS:
        seen = {}
        for v in values:
            t = gvl.gvl_tuning.from_buffer_copy(best)
            put(t, field, b, v)
            try:
                gvl.gvl_set_tuning(c, t)
            except gvl.GvlError:
                continue  # not a valid combination with the other limits
            seen[v] = measure()
        gvl.gvl_set_tuning(c, best)
        if not seen:
            continue
        v_best = min(seen, key=seen.get)
        if seen[v_best] < (1.0 - MIN_GAIN) * cur and v_best != get(best, field, b):
            put(best, field, b, v_best)
            cur = seen[v_best]
        name = field + ("[%d]" % b if b is not None else "")
        line = "  %s: %s -> %s" % (name, ", ".join("%s %.2f ms" % (v, ms) for v, ms in sorted(seen.items())),
                                   get(best, field, b))
        notes.append(line)
        log(line)
    gvl.gvl_set_tuning(c, best)
    final = measure()
    notes.append("  tuned %.2f ms (default %.2f ms, %.1f %%)" % (final, base, 100.0 * (final - base) / base))
    log(notes[-1])
    return best, notes


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--classes", default="small,lowdeg,skewed,batch")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=os.path.join(HERE, "tune.txt"))
    args = ap.parse_args()
    os.environ.setdefault("GVL_TUNE_FILE", "none")  # tune from the compiled defaults
    log = lambda s: print(s, flush=True)  # noqa: E731
    lines = ["# Launch shapes per class of graph, written by paper_2312_13936_amd/tune.py on one MI355X.",
             "# <class> bin_max[0..5] decide_grid commit_grid agg_grid"]
    body = []
    for cls in args.classes.split(","):
        t, notes = tune(cls, args.reps, log)
        lines += ["# " + n for n in notes]
        body.append("%s %s %d %d %d" % (cls, " ".join(str(x) for x in t.bin_max), t.decide_grid, t.commit_grid,
                                         t.agg_grid))
    with open(args.out, "w") as f:
        f.write("\n".join(lines + body) + "\n")
    log("wrote " + args.out)


if __name__ == "__main__":
    main()
