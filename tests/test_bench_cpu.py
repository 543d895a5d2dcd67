"""Host logic of the benchmark, CPU only: the one-GPU refusal, the counter summary (calibration by
the copy kernels, per-family bytes per launch), the staleness check of the committed summary and
the roofline arithmetic."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import datagen  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for d, (name, grid, vals) in enumerate(rows):
            for v in vals:  # one row per hardware instance, summed per dispatch
                w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter,
                            "Counter_Value": v})


def test_summarize_traffic_calibrates_by_the_copies(tmp_path):
    mib = 4
    copy = "__amd_rocclr_copyBuffer"
    relin = "void cw::k_relin_f<cw::Shape<13, 3, 5, 3, 3, 3, 2, 2>, true>(args)"
    # the copies' FETCH_SIZE reads half of what moved (factor 2), WRITE_SIZE all of it (factor 1);
    # a smaller copy dispatch of another grid must not enter the calibration
    fetch = [(copy, 4096, [mib * 1024 / 4] * 2)] * 3 + [(copy, 64, [1.0])] + \
            [(relin, 2621440, [100.0, 50.0])] * 4 + [(relin, 1310720, [10.0])] * 2
    write = [(copy, 4096, [mib * 1024 / 2] * 2)] * 3 + [(copy, 64, [1.0])] + \
            [(relin, 2621440, [30.0])] * 4 + [(relin, 1310720, [5.0])] * 2
    fcsv, wcsv, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "t.json"
    _counter_csv(fcsv, "FETCH_SIZE", fetch)
    _counter_csv(wcsv, "WRITE_SIZE", write)
    bench.summarize_traffic(str(fcsv), str(wcsv), mib, "mid", 16384, 8,
                            {"chunk_elems": 512, "query_group": 1, "relin_group": 0}, str(out))
    d = json.load(open(out))
    assert d["fetch_factor"] == pytest.approx(2.0) and d["write_factor"] == pytest.approx(1.0)
    r = d["families"]["relin"]
    assert r["grid_size"] == 2621440 and r["dispatches"] == 4  # the most-dispatched launch shape
    assert r["bytes_per_launch"] == pytest.approx((150.0 * 2 + 30.0) * 1024)
    assert d["workload"] == "mid" and d["n"] == 16384 and d["batch"] == 8


def test_traffic_table_is_null_when_stale(tmp_path, monkeypatch):
    cfg = datagen.CONFIGS["mid"]
    sched = {"chunk_elems": 512, "query_group": 1, "relin_group": 0}
    fcsv, wcsv, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "t.json"
    _counter_csv(fcsv, "FETCH_SIZE", [("copyBuffer", 1, [512.0])] * 3 + [("k_scale<5, 5>", 9, [8.0])])
    _counter_csv(wcsv, "WRITE_SIZE", [("copyBuffer", 1, [1024.0])] * 3 + [("k_scale<5, 5>", 9, [4.0])])
    bench.summarize_traffic(str(fcsv), str(wcsv), 1, cfg.name, cfg.n, 8, sched, str(out))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    table = bench.traffic_table(cfg, cfg.n, 8, dict(sched, ns_per_elem=0.0))
    assert table["scale"]["bytes_per_launch"] == pytest.approx((8.0 * 2 + 4.0) * 1024)
    assert bench.traffic_table(cfg, cfg.n, 4, sched) is None                       # other batch size
    assert bench.traffic_table(cfg, cfg.n, 8, dict(sched, chunk_elems=256)) is None  # other schedule
    d = json.load(open(out))
    d["kernel_source_sha256"] = "0" * 64                                            # other kernels
    json.dump(d, open(out, "w"))
    assert bench.traffic_table(cfg, cfg.n, 8, sched) is None


def test_roofline_arithmetic():
    bfly = 53248.0
    prof = {"relin": (600.0, 100, 100 * 35 * 512 * bfly), "scale": (300.0, 100, 1.0)}
    traffic = {"relin": {"bytes_per_launch": 1.2e9}}
    r = bench.roofline(prof, 2, True, traffic)
    assert r["kernel"] == "relin" and r["avg_launch_ms"] == pytest.approx(6.0)
    achieved = 35 * 512 * bfly / 6e-3
    peak = 78.6e12 / 2 / 8  # fp64 instructions per second over 8 per butterfly
    assert r["achieved"] == pytest.approx(achieved / 1e12) and r["peak"] == pytest.approx(peak / 1e12)
    assert r["frac"] == pytest.approx(achieved / peak)
    assert r["traffic"] == 1.2e9 and r["hbm_GBps_at_traffic"] == pytest.approx(1.2e9 / 6e-3 / 1e9)
    assert r["launches_per_step"] == 50
    assert bench.roofline(prof, 2, True, None)["traffic"] is None
    # every family: its fraction of the butterfly roof (transforms) and of HBM (where counted)
    fam = r["families"]
    assert fam["relin"]["alu_frac"] == pytest.approx(achieved / peak)
    assert fam["relin"]["hbm_GBps"] == pytest.approx(1.2e9 / 6e-3 / 1e9)
    assert fam["relin"]["hbm_frac"] == pytest.approx(1.2e9 / 6e-3 / 8e12)
    assert "alu_frac" not in fam["scale"] and "hbm_frac" not in fam["scale"]
