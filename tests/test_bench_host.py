"""Host-side pieces of bench.py's measurement (no GPU): the kernel identity
code, the committed HBM-traffic record and its source-hash guard, and the
selection of profiler rows by the boot-clock windows the benchmark prints."""
import csv
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_kernel_name_codes(bench):
    # precision x 8 + (f64 output) x 4 + A k-contiguous x 2 + B k-contiguous
    assert bench.kernel_name(1 * 8 + 4 + 2 + 1) == "ftd::gemm_kernel<float, double, true, true>"
    assert bench.kernel_name(1 * 8 + 2) == "ftd::gemm_kernel<float, float, true, false>"
    assert bench.kernel_name(0 * 8 + 4 + 1) == "ftd::gemm_kernel<double, double, false, true>"


def test_traffic_record_matches_current_source(bench):
    path = os.path.join(ROOT, "profiles", "traffic_hp_n21_loc4_nl1_d10_D128_T300.json")
    rec = json.load(open(path))
    t = bench.measured_traffic(rec["kernel"], rec["workload"])
    # the committed record was taken with the committed GEMM source
    assert t is not None and t == pytest.approx(rec["traffic_bytes_per_launch"])
    # its own arithmetic: counters in KiB, scaled by the copy calibration
    fb = rec["fetch_size_kib_in_window"] * 1024 * rec["fetch_factor"] / rec["dispatches_in_window"]
    wb = rec["write_size_kib_in_window"] * 1024 * rec["write_factor"] / rec["dispatches_in_window"]
    assert fb + wb == pytest.approx(rec["traffic_bytes_per_launch"], rel=1e-12)
    copy_kib = rec["calibration_copy_bytes"] / 1024
    assert rec["fetch_factor"] == pytest.approx(copy_kib / rec["fetch_size_kib_for_copy"])
    assert bench.measured_traffic("some other kernel", rec["workload"]) is None
    assert bench.measured_traffic(rec["kernel"], "another workload") is None


def test_window_selection(bench, tmp_path, capsys):
    log = tmp_path / "err"
    ms = 1000000   # timestamps in ns
    log.write_text(f"[bench] timed region boottime_ns {100 * ms} {200 * ms}\n"
                   f"[bench] calibration copy of 1024 bytes boottime_ns {300 * ms} {310 * ms}\n")
    rows = [("k_a", 90 * ms, 95 * ms), ("k_a", 100 * ms, 150 * ms), ("k_b", 120 * ms, 160 * ms),
            ("k_a", 200 * ms, 260 * ms), ("copy", 305 * ms, 309 * ms), ("k_b", 400 * ms, 410 * ms)]
    f = tmp_path / "trace.csv"
    with open(f, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for r in rows:
            w.writerow(r)
    bench.summarize("trace", str(f), str(log))
    out = capsys.readouterr().out
    # dispatches that start inside [100, 200]: k_a at 100 and 200, k_b at 120
    assert "[timed steps] window 0.100 s, dispatches in window 3" in out
    assert "[calibration copy] window 0.010 s, dispatches in window 1" in out
    line = [l for l in out.splitlines() if l.endswith("\tk_a")][0]
    calls, total_ms = line.split("\t")[:2]
    assert calls == "2" and float(total_ms) == pytest.approx(50 + 60)
