"""Host logic of the benchmark (no GPU): the rocprofv3 counter summary that
turns FETCH_SIZE / WRITE_SIZE readings into HBM bytes per launch, the check
that a stored summary belongs to the current kernel source, and the
single-GPU guard."""

import csv
import json
import os
import subprocess
import sys

import pytest

import bench

KIB = 1024.0
MIXED = "void mfmg::k_smooth<float, float, __half, 256, 0>(mfmg::LevelArgs<float, float, __half>, int)"
FP64 = "void mfmg::k_smooth<double, double, double, 2, 0>(mfmg::LevelArgs<double, double, double>, int)"
COPY = "__amd_rocclr_copyBuffer"


def write_counters(path, counter, rows):
    """rows: (dispatch id, kernel name, [KiB per counter instance])."""
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                           "Counter_Value"])
        w.writeheader()
        for d, name, vals in rows:
            for v in vals:
                w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter,
                            "Counter_Value": v})


def cycle_kernels(smooth_name):
    """Kernel names of one V-cycle's dispatches (a short one) and the KiB of
    each: fill, two half-sweeps, restriction, bottom, prolongation, two
    half-sweeps."""
    t = smooth_name.replace("k_smooth<", "{}<")
    return [("void mfmg::k_fill<float>(float*, long, float)", 10.0),
            (smooth_name, 100.0), (smooth_name, 100.0),
            (t.format("k_restrict"), 50.0), (t.format("k_bottom"), 5.0),
            (t.format("k_prolong"), 20.0), (smooth_name, 100.0), (smooth_name, 100.0)]


CYCLE_KIB = 485.0


def counter_run(tmp_path, counter, smooth_name, smooth_kib, copy_kib, copies=4, tag=""):
    """One counter pass as the traffic pass lays it out: a small copy, five
    half-sweeps (each reported as two counter instances), five cycles, then
    the 1 GiB copies that scale the counter."""
    rows = [(1, COPY, [64.0])]
    rows += [(2 + i, smooth_name, [smooth_kib / 2, smooth_kib / 2]) for i in range(5)]
    d = 7
    for _ in range(5):
        for name, kib in cycle_kernels(smooth_name):
            rows.append((d, name, [kib]))
            d += 1
    rows += [(d + i, COPY, [copy_kib]) for i in range(copies)]
    path = os.path.join(tmp_path, f"{counter}{tag}.csv")
    write_counters(path, counter, rows)
    return path


def test_summary_scales_each_counter_by_its_copy_reading(tmp_path):
    f = counter_run(tmp_path, "FETCH_SIZE", MIXED, 3000.0, bench.COPY_BYTES / 2 / KIB)
    w = counter_run(tmp_path, "WRITE_SIZE", MIXED, 500.0, bench.COPY_BYTES / KIB)
    prec, rec = bench.summarize_pmc(f, w, 10)
    assert prec == "mixed"
    assert rec["level"] == 10
    assert rec["counters"]["FETCH_SIZE"]["copy_factor"] == pytest.approx(0.5)
    assert rec["counters"]["WRITE_SIZE"]["copy_factor"] == pytest.approx(1.0)
    assert rec["counters"]["FETCH_SIZE"]["launches"] == 5
    assert rec["fetch_bytes_per_launch"] == pytest.approx(3000.0 * KIB / 0.5)
    assert rec["write_bytes_per_launch"] == pytest.approx(500.0 * KIB)
    assert rec["hbm_bytes_per_launch"] == pytest.approx(6000.0 * KIB + 500.0 * KIB)
    # the cycles: every cycle kernel after the first fill, per bottom dispatch
    assert rec["counters"]["FETCH_SIZE"]["cycles"] == 5
    assert rec["cycle_fetch_bytes"] == pytest.approx(CYCLE_KIB * KIB / 0.5)
    assert rec["cycle_hbm_bytes"] == pytest.approx(CYCLE_KIB * KIB / 0.5 + CYCLE_KIB * KIB)


def test_summary_names_the_fp64_hierarchy(tmp_path):
    f = counter_run(tmp_path, "FETCH_SIZE", FP64, 6000.0, bench.COPY_BYTES / 2 / KIB)
    w = counter_run(tmp_path, "WRITE_SIZE", FP64, 1000.0, bench.COPY_BYTES / KIB)
    prec, rec = bench.summarize_pmc(f, w, 10)
    assert prec == "fp64"
    assert rec["hbm_bytes_per_launch"] == pytest.approx(13000.0 * KIB)


def test_summary_refuses_mixed_hierarchies_and_missing_copies(tmp_path):
    f = counter_run(tmp_path, "FETCH_SIZE", MIXED, 3000.0, bench.COPY_BYTES / 2 / KIB)
    w64 = counter_run(tmp_path, "WRITE_SIZE", FP64, 500.0, bench.COPY_BYTES / KIB)
    with pytest.raises(SystemExit):
        bench.summarize_pmc(f, w64, 10)
    w3 = counter_run(tmp_path, "WRITE_SIZE", MIXED, 500.0, bench.COPY_BYTES / KIB, copies=3,
                     tag="_3")
    with pytest.raises(SystemExit):
        bench.summarize_pmc(f, w3, 10)


def test_stored_traffic_is_used_only_for_its_source_and_level(tmp_path, monkeypatch):
    os.makedirs(os.path.join(tmp_path, "profiles"))
    rec = {"source_hash": "h-current", "level": 10, "hbm_bytes_per_launch": 123.0}
    with open(os.path.join(tmp_path, "profiles", "traffic_smooth_large_workload.json"), "w") as fh:
        json.dump({"mixed": rec}, fh)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "h-current")
    assert bench.measured_traffic("mixed", 10) == 123.0
    assert bench.measured_traffic("mixed", 9) is None
    assert bench.measured_traffic("fp64", 10) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "h-edited")
    assert bench.measured_traffic("mixed", 10) is None


def test_committed_traffic_records_are_consistent():
    path = os.path.join(bench.ROOT, "profiles", "traffic_smooth_large_workload.json")
    with open(path) as fh:
        store = json.load(fh)
    assert "mixed" in store
    for rec in store.values():
        assert rec["hbm_bytes_per_launch"] == pytest.approx(
            rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"])
        for c in rec["counters"].values():
            assert c["per_launch_bytes"] == pytest.approx(
                c["per_launch_bytes_raw"] / c["copy_factor"])


def test_trace_summary_keeps_kernel_averages_with_the_source(tmp_path, monkeypatch):
    os.makedirs(os.path.join(tmp_path, "profiles"))
    stats = os.path.join(tmp_path, "kernel_stats.csv")
    with open(stats, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs",
                                           "Percentage", "MinNs", "MaxNs", "StdDev"])
        w.writeheader()
        w.writerow({"Name": MIXED, "Calls": 4,
                    "TotalDurationNs": 440000, "AverageNs": 110000.0, "Percentage": 50,
                    "MinNs": 100000, "MaxNs": 120000, "StdDev": 1})
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "h-current")
    bench.summarize_trace(stats)
    assert bench.traced_launch_us("mfmg::k_smooth<float, float, __half, 256, 0>") == 110.0
    assert bench.traced_launch_us("mfmg::k_restrict<float, float, __half, 2>") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "h-edited")
    assert bench.traced_launch_us("mfmg::k_smooth<float, float, __half, 256, 0>") is None


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
