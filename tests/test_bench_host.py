"""Host logic of the measurement tools (no GPU needed).

bench.py must refuse more than one GPU before it touches a device, and the
profile summaries must scale the rocprofv3 byte counters by what they read
for a copy of known size and stop vouching for them once the kernel
sources change.
"""
import csv
import json
import os
import subprocess
import sys

import pytest

from paper_2312_13936_amd import profile_summary as ps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}), ([], {"WORLD_SIZE": "4"})])
def test_bench_refuses_more_than_one_gpu(argv, env):
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, capture_output=True, text=True,
                       env=e, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, v in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def test_counters_scale_by_the_copy_and_sum_per_class(tmp_path):
    calib = 1 << 30
    # the copy reads half its bytes in counted KiB, writes all of them
    fetch = [("__amd_rocclr_copyBuffer", calib / 1024 / 2),
             ("void gvl::k_decide_wide<float, 0, false>(...)", 1000.0),
             ("void gvl::k_hub_part_eval<float, 1, false>(...)", 500.0),
             ("void gvl::k_agg_rows<float, float, 256, 2048>(...)", 300.0),
             ("void gvl::k_gagg_gather<float>(...)", 100.0),
             ("gvl::k_mod_squares(...)", 7777.0)]          # neither class
    write = [("__amd_rocclr_copyBuffer", calib / 1024),
             ("void gvl::k_decide_groups<float, 0, false>(...)", 10.0),
             ("void gvl::k_agg_group<float, float, 4, 3>(...)", 20.0)]
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    _counter_csv(fp, "FETCH_SIZE", fetch)
    _counter_csv(wp, "WRITE_SIZE", write)
    out = tmp_path / "c.md"
    ps.counters(str(fp), str(wp), str(calib), "2", str(out), "cmd")  # the run made two calls
    rec = ps.recorded_traffic(str(out))
    assert rec is not None and rec["digest"] == ps.source_digest() and rec["calls"] == 2
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["scan_fetch_bytes"] == pytest.approx(1500.0 * 1024 * 2 / 2)
    assert rec["agg_fetch_bytes"] == pytest.approx(400.0 * 1024 * 2 / 2)
    assert rec["scan_write_bytes"] == pytest.approx(10.0 * 1024 / 2)
    assert rec["agg_write_bytes"] == pytest.approx(20.0 * 1024 / 2)


def test_recorded_traffic_is_dropped_when_sources_change(tmp_path):
    rec = {"digest": "0" * 16, "calib_bytes": 1, "fetch_scale": 1.0, "write_scale": 1.0,
           "scan_fetch_bytes": 1.0, "scan_write_bytes": 1.0, "agg_fetch_bytes": 1.0, "agg_write_bytes": 1.0}
    p = tmp_path / "stale.md"
    p.write_text("# x\n\ncounters-json: " + json.dumps(rec) + "\n")
    assert ps.source_digest() != "0" * 16
    assert ps.recorded_traffic(str(p)) is None
    assert ps.recorded_traffic(str(tmp_path / "missing.md")) is None



def test_pmc_tables_per_call_totals_and_ratios(tmp_path):
    a, b = tmp_path / "a.csv", tmp_path / "b.csv"
    scan = "void gvl::k_decide_groups<float, 0, false>(...)"
    agg = "void gvl::k_agg_rows<float, float, 256, 2048>(...)"
    _counter_csv(a, "SQ_WAVE_CYCLES", [(scan, 1000.0), (agg, 400.0)])
    with open(a, "a", newline="") as f:  # a second counter of the same pass
        csv.writer(f).writerows([[scan, "SQ_WAIT_ANY", 700.0], [agg, "SQ_WAIT_ANY", 100.0]])
    _counter_csv(b, "TCC_EA0_RDREQ_sum", [(scan, 50.0), (agg, 20.0)])
    with open(b, "a", newline="") as f:
        csv.writer(f).writerows([[scan, "TCC_EA0_RDREQ_LEVEL_sum", 45000.0], [agg, "TCC_EA0_RDREQ_LEVEL_sum", 16000.0]])
    out = tmp_path / "p.md"
    ps.pmc("2", str(out), "cmd", str(a), str(b))  # two calls: totals halved
    text = out.read_text()
    totals, derived = text.split("Derived")
    rows = {l.split("|")[1].strip(): [c.strip() for c in l.split("|")[2:-1]] for l in totals.splitlines()
            if l.startswith("| **") or l.startswith("| `")}
    # table of totals: SQ_WAVE_CYCLES, SQ_WAIT_ANY, TCC_EA0_RDREQ_sum, TCC_EA0_RDREQ_LEVEL_sum per call
    assert rows["**neighbour-community scan**"][:4] == ["500", "350", "25", "2.25e+04"]
    assert rows["**aggregation rows**"][:4] == ["200", "50", "10", "8e+03"]
    # waiting fraction and mean latency are ratios of the per-call totals
    assert "| **neighbour-community scan** | 0.7 | 900 |" in derived
    assert "| **aggregation rows** | 0.25 | 800 |" in derived
    assert "Kernel sources digest: %s" % ps.source_digest() in text
