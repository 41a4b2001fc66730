"""bench.py's trace summaries (host-only: synthetic rocprofv3 CSV files)."""
import csv
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _write_trace(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "x_kernel_trace.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for name, a, b in rows:
            w.writerow({"Kernel_Name": name, "Start_Timestamp": a, "End_Timestamp": b})


def test_summarize_gaps_busy_fraction_and_grouping(tmp_path):
    # kernels (ns): [0, 100 us], overlapping [50 us, 150 us], gap of 50 us, [200 us, 300 us],
    # gap of 10 us (below the 20 us floor), [310 us, 400 us], gap of 100 us, [500 us, 600 us]
    us = 1000
    rows = [("void gcge::k_a<double, 2>(long, double*)", 0, 100 * us),
            ("void gcge::k_b(long)", 50 * us, 150 * us),
            ("__amd_rocclr_copyBuffer", 200 * us, 300 * us),
            ("void gcge::k_a<double, 2>(long, double*)", 310 * us, 400 * us),
            ("__amd_rocclr_copyBuffer", 500 * us, 600 * us)]
    d = str(tmp_path / "trace")
    _write_trace(d, rows)
    out = bench.summarize_gaps(d)
    # busy: 150 + 100 + 90 + 100 = 440 of a 600 us span
    assert "kernels busy 0.4 ms (73.3 %)" in out
    assert "gaps over 20 us: 0.1 ms in 2" in out
    assert "| `k_b` → `__amd_rocclr_copyBuffer` | 1 | 0.1 | 50.0 |" in out
    assert "| `k_a<double, 2>` → `__amd_rocclr_copyBuffer` | 1 | 0.1 | 100.0 |" in out
    assert "k_a<double, 2>` → `k_b" not in out   # overlapping dispatches leave no gap


def test_short_name():
    assert bench.short_name("void gcge::k_spmms<double, 32, 2, 0, 2>(long, int const*)") == \
        "k_spmms<double, 32, 2, 0, 2>"
    assert bench.short_name("gcge::(anonymous namespace)::k_tridiag<8, 1, 4>(int, double*)") == "k_tridiag<8, 1, 4>"
