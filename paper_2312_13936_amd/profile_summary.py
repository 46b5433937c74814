"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_2312_13936_amd.profile_summary stats  <kernel_stats.csv> <bench.json> <calls> <out.md> <command>
    python -m paper_2312_13936_amd.profile_summary counters <fetch.csv> <write.csv> <calib_bytes> <calls> <out.md> <command>
    python -m paper_2312_13936_amd.profile_summary pmc <calls> <out.md> <command> <counter_collection.csv>...

`stats` writes the per-kernel time table of a `--kernel-trace --stats` run
(`calls` gvl_leiden calls) grouped into the scan and aggregation classes,
per call beside the bench line's HIP-event times.  `counters` sums FETCH_SIZE
and WRITE_SIZE (KiB per dispatch) over the dispatches of each class, divides
by the number of gvl_leiden calls the run made, scales each counter by what
it reads for the device-to-device copy of `calib_bytes` bytes that the
benchmark runs first, and records the result with a digest of the kernel
sources; bench.py reports it as the roofline's `traffic` only while that
digest matches the current sources.  `pmc` tabulates any other counters
(one csv per rocprofv3 pass) per call, by kernel class and for the kernels
that take the most time.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import re
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
SCAN = re.compile(r"k_decide_|k_hub_(gather|eval|part_eval)")
AGG = re.compile(r"k_agg_(group|rows)|k_gagg_|k_member_degrees")
COPY = re.compile(r"copyBuffer|copy_kernel|CatArrayBatchedCopy|elementwise_kernel.*copy", re.I)


def source_digest() -> str:
    """sha256 (16 hex digits) over the HIP sources of libgvl.so."""
    h = hashlib.sha256()
    d = os.path.join(_HERE, "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def short(name: str) -> str:
    name = re.sub(r"gvl::", "", name)
    name = re.sub(r"GraphView<([a-z]+)>", r"GV<\1>", name)
    return name


def stats(stats_csv, bench_json, calls, out, command):
    calls = int(calls)
    rows = list(csv.DictReader(open(stats_csv)))
    bench = json.loads(open(bench_json).read().strip().splitlines()[-1])
    tot = sum(float(r["TotalDurationNs"]) for r in rows) / 1e6
    cls = collections.defaultdict(float)
    for r in rows:
        ms = float(r["TotalDurationNs"]) / 1e6
        if SCAN.search(r["Name"]):
            cls["scan"] += ms
        elif AGG.search(r["Name"]):
            cls["agg"] += ms
    ph = bench.get("phases", {})
    lines = ["# Kernel time summary: %s" % bench["config"]["workload"], "",
             "Command (from the repository root on the MI355X box):", "", "```", command, "```", "",
             "One gvl_leiden call: %.1f ms wall, Q = %.4f, %d passes, %s mode." % (
                 bench["ms_per_step"], bench["modularity"], bench["passes"], bench["config"]["mode"]), "",
             "| kernel class | rocprofv3, per call (ms) | HIP events in bench.py, per call (ms) |", "|---|---|---|",
             "| neighbour-community scan (`k_decide_*`, `k_hub_gather/eval/part_eval`) | %.1f | %.1f |" % (
                 cls["scan"] / calls, ph.get("scan_kernels_ms", float("nan"))),
             "| aggregation rows (`k_agg_*`, `k_gagg_*`, `k_member_degrees`) | %.1f | %.1f |" % (
                 cls["agg"] / calls, ph.get("agg_kernels_ms", float("nan"))),
             "| all kernels | %.1f | |" % (tot / calls), "",
             "Per call = the run's total over its %d gvl_leiden calls.  The HIP-event spans bracket every" % calls,
             "launch of a class and the short gaps between them.  The table below is the whole run.", "",
             "| total ms | calls | avg us | % | kernel |", "|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:25]:
        lines.append("| %.2f | %s | %.1f | %.1f | `%s` |" % (
            float(r["TotalDurationNs"]) / 1e6, r["Calls"], float(r["AverageNs"]) / 1e3, float(r["Percentage"]),
            short(r["Name"])[:110]))
    lines.append("")
    lines.append("Kernel sources digest: %s" % source_digest())
    open(out, "w").write("\n".join(lines) + "\n")


def _sum(path, counter):
    per = collections.defaultdict(float)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            per[r["Kernel_Name"]] += float(r["Counter_Value"])
    return per


def counters(fetch_csv, write_csv, calib_bytes, calls, out, command):
    calib_bytes = int(calib_bytes)
    calls = int(calls)
    f = _sum(fetch_csv, "FETCH_SIZE")
    w = _sum(write_csv, "WRITE_SIZE")
    fc = [v for k, v in f.items() if COPY.search(k)]
    wc = [v for k, v in w.items() if COPY.search(k)]
    if not fc or not wc:
        raise SystemExit("no copy kernel found for the calibration")
    kf = calib_bytes / (max(fc) * 1024.0)   # bytes per counted KiB
    kw = calib_bytes / (max(wc) * 1024.0)
    res = {"digest": source_digest(), "calib_bytes": calib_bytes, "calls": calls, "fetch_scale": kf,
           "write_scale": kw}
    for name, rx in (("scan", SCAN), ("agg", AGG)):
        fb = sum(v for k, v in f.items() if rx.search(k)) * 1024.0 * kf / calls
        wb = sum(v for k, v in w.items() if rx.search(k)) * 1024.0 * kw / calls
        res[name + "_fetch_bytes"] = fb
        res[name + "_write_bytes"] = wb
    lines = ["# HBM traffic of the Leiden kernel classes (rocprofv3 counters)", "",
             "Commands (from the repository root on the MI355X box), one counter per run:", "", "```",
             command, "```", "",
             "FETCH_SIZE and WRITE_SIZE are summed over the dispatches of each class, divided by the",
             "%d gvl_leiden calls of the run (bytes per call) and" % calls,
             "scaled by what each counter reads for a device-to-device copy of %d bytes run first" % calib_bytes,
             "(fetch x%.4f, write x%.4f per counted byte)." % (kf, kw), "",
             "| class | fetched (GB) | written (GB) |", "|---|---|---|",
             "| neighbour-community scan | %.2f | %.2f |" % (res["scan_fetch_bytes"] / 1e9,
                                                             res["scan_write_bytes"] / 1e9),
             "| aggregation rows | %.2f | %.2f |" % (res["agg_fetch_bytes"] / 1e9, res["agg_write_bytes"] / 1e9),
             "", "counters-json: " + json.dumps(res), ""]
    open(out, "w").write("\n".join(lines))


def pmc(calls, out, command, *csvs):
    """Per-call totals of every counter in the given counter_collection.csv
    files, by kernel class and for the 12 kernels with the largest
    SQ_BUSY_CYCLES (or the first counter)."""
    calls = int(calls)
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    names = []
    for path in csvs:
        for r in csv.DictReader(open(path)):
            c = r["Counter_Name"]
            if c not in names:
                names.append(c)
            per[short(r["Kernel_Name"].split("(")[0]).replace("void ", "")][c] += float(r["Counter_Value"]) / calls
    key = "SQ_BUSY_CYCLES" if "SQ_BUSY_CYCLES" in names else names[0]
    cls = collections.defaultdict(lambda: collections.defaultdict(float))
    for k, v in per.items():
        for name, rx in (("neighbour-community scan", SCAN), ("aggregation rows", AGG)):
            if rx.search(k):
                for c, x in v.items():
                    cls[name][c] += x
    def row(label, v):
        return "| %s | " % label + " | ".join("%.3g" % v.get(c, 0.0) for c in names) + " |"
    lines = ["# Hardware counters per gvl_leiden call (rocprofv3 --pmc)", "",
             "Commands (from the repository root on the MI355X box), one pass per counter group:", "", "```",
             command, "```", "", "Totals per call (the run made %d calls)." % calls, "",
             "| kernel / class | " + " | ".join(names) + " |", "|---" * (len(names) + 1) + "|"]
    for name in ("neighbour-community scan", "aggregation rows"):
        lines.append(row("**%s**" % name, cls[name]))
    top = sorted(per, key=lambda k: -per[k].get(key, 0.0))[:12]
    for k in top:
        lines.append(row("`%s`" % k[:70], per[k]))
    # ratios of counter pairs that were both collected
    ratios = [("L2 hit rate", "TCC_HIT_sum", ("TCC_HIT_sum", "TCC_MISS_sum")),
              ("wave-cycles waiting", "SQ_WAIT_ANY", ("SQ_WAVE_CYCLES",)),
              ("wave-cycles waiting to issue", "SQ_WAIT_INST_ANY", ("SQ_WAVE_CYCLES",)),
              ("mean EA read latency (cycles)", "TCC_EA0_RDREQ_LEVEL_sum", ("TCC_EA0_RDREQ_sum",)),
              ("mean EA write latency (cycles)", "TCC_EA0_WRREQ_LEVEL_sum", ("TCC_EA0_WRREQ_sum",)),
              ("mean EA atomic latency (cycles)", "TCC_EA0_ATOMIC_LEVEL_sum", ("TCC_EA0_ATOMIC_sum",))]
    ratios = [r for r in ratios if r[1] in names and all(c in names for c in r[2])]
    if ratios:
        def ratio(v, num, den):
            d = sum(v.get(c, 0.0) for c in den)
            return "%.3g" % (v.get(num, 0.0) / d) if d > 0 else "-"
        lines += ["", "Derived (ratios of the totals above):", "",
                  "| kernel / class | " + " | ".join(r[0] for r in ratios) + " |", "|---" * (len(ratios) + 1) + "|"]
        for label, v in [("**%s**" % n, cls[n]) for n in ("neighbour-community scan", "aggregation rows")] + \
                        [("`%s`" % k[:70], per[k]) for k in top]:
            lines.append("| %s | " % label + " | ".join(ratio(v, r[1], r[2]) for r in ratios) + " |")
    lines += ["", "Kernel sources digest: %s" % source_digest(), ""]
    open(out, "w").write("\n".join(lines))


def recorded_traffic(path):
    """The counters-json record of a counters summary, or None if the file is
    missing or the kernel sources changed since it was taken."""
    try:
        for line in open(path):
            if line.startswith("counters-json: "):
                rec = json.loads(line[len("counters-json: "):])
                return rec if rec.get("digest") == source_digest() else None
    except OSError:
        return None
    return None


if __name__ == "__main__":
    if len(sys.argv) >= 7 and sys.argv[1] == "stats":
        stats(*sys.argv[2:7])
    elif len(sys.argv) >= 8 and sys.argv[1] == "counters":
        counters(*sys.argv[2:8])
    elif len(sys.argv) >= 6 and sys.argv[1] == "pmc":
        pmc(*sys.argv[2:])
    else:
        print(__doc__)
        sys.exit(2)
