"""Host logic of bench.py (no GPU): the one-GPU contract, the HBM counter summary's scaling by the
calibration copy, and the stored traffic figure's tie to the sweep sources."""
import csv
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr and r.stdout == ""


def _counter_csv(path, name, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (kernel, grid, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": kernel, "Grid_Size": grid, "Counter_Name": name,
                        "Counter_Value": value})


def test_counter_summary_scales_by_the_calibration_copy(tmp_path):
    # the copy reads and writes 1 GiB; FETCH_SIZE reports half of it, WRITE_SIZE all of it (KiB)
    sweep = "void top::sweep_kernel<float, 3, 3, true, true, 512, false>(top::SweepArgs<float>)"
    copy = "void at::native::vectorized_elementwise_kernel<4, at::native::MulFunctor<float>>"
    probe = (sweep, 100, 1.0)                 # an autotune probe at another grid: not counted
    f, w = tmp_path / "pf.csv", tmp_path / "pw.csv"
    _counter_csv(f, "FETCH_SIZE", [probe, (copy, 1, 524288.0), (sweep, 5, 1000.0), (sweep, 5, 1002.0), (sweep, 5, 998.0)])
    _counter_csv(w, "WRITE_SIZE", [probe, (copy, 1, 1048576.0), (sweep, 5, 700.0), (sweep, 5, 700.0)])
    md = bench.counters_summary(str(f), str(w))
    kv = dict(l.split(" = ", 1) for l in md.splitlines() if " = " in l)
    expect = 1000.0 * 1024 * 2.0 + 700.0 * 1024 * 1.0
    assert abs(float(kv["traffic_bytes_per_launch"]) - expect) <= 1e-6 * expect
    assert kv["sweep_source_digest"].strip() == bench.sweep_source_digest()


def test_stored_traffic_needs_the_current_sources(tmp_path, monkeypatch):
    md = tmp_path / "c.md"
    md.write_text(f"traffic_bytes_per_launch = 1.5e+09\nsweep_source_digest = {bench.sweep_source_digest()}\n")
    monkeypatch.setattr(bench, "COUNTERS_MD", str(md))
    assert bench.stored_traffic() == pytest.approx(1.5e9)
    md.write_text("traffic_bytes_per_launch = 1.5e+09\nsweep_source_digest = 0000000000000000\n")
    assert bench.stored_traffic() is None
