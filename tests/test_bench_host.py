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
    assert bench.kernel_name(2 * 8 + 4 + 2 + 1) == "ftd::gemm_bx3_kernel<double, true, true>"


def test_error_and_window_mobility(bench):
    import numpy as np
    ref = np.array([1.0 + 0.1j, 0.5, 0.25])
    C = ref + np.array([0.0, 1e-5, -2e-5j])
    assert bench.c_err(C, ref, 2.0) == pytest.approx(1e-5)
    # trapezoid of Re C over [0, 3 dt] with C(0) = c0 prepended
    mu = bench.mu_window(ref, 0.5, 2.0, 2.0)
    assert mu == pytest.approx(2.0 * 0.5 * (1.0 + 1.0 + 0.5 + 0.125))


def test_roofline_entries(bench):
    st = {k: [0] * 32 for k in ("kind_launches", "kind_ms", "kind_flops", "kind_bytes")}
    st["kind_launches"][13], st["kind_ms"][13], st["kind_flops"][13] = 10, 2.0, 1.5e11
    st["kind_launches"][10], st["kind_ms"][10], st["kind_flops"][10] = 4, 1.0, 5e10
    out = bench.roofline_entries(st, lambda k: 157.3)
    assert [e["kernel"] for e in out] == ["ftd::gemm_kernel<float, double, false, true>",
                                          "ftd::gemm_kernel<float, float, true, false>"]
    assert out[0]["achieved"] == pytest.approx(75.0) and out[0]["avg_launch_ms"] == 0.2
    assert out[1]["frac"] == pytest.approx(50.0 / 157.3)


def test_cpu_baseline_assembles_a_step(bench):
    """Every distinct site shape is timed once and the step is the sum over
    both states' sites; a larger Krylov count can only make it slower."""
    from paper_2003_13245_amd import workloads as W
    from oracle import model as Mdl
    wl = W.rubrene_shaped(n_mol=3, n_loc=1, n_nl=1, levels=3, D=6)
    L = len(Mdl.site_dims(wl.model))
    bonds = [min(6, 4 ** (i + 1), 4 ** (L - 1 - i)) for i in range(L - 1)]
    a = bench.cpu_baseline(wl, [bonds, bonds], 4.0, rep_s=0.01)
    b = bench.cpu_baseline(wl, [bonds, bonds], 8.0, rep_s=0.01)
    assert a["kind"] == "oracle" and a["unit"] == "pair-steps/s" and a["cores"] >= 1
    assert a["value"] > 0 and b["seconds_per_pair_step"] > a["seconds_per_pair_step"] * 1.2


def test_traffic_record_matches_current_source(bench):
    path = os.path.join(ROOT, "profiles", "traffic_hp_n21_loc4_nl1_d10_D128_T300.json")
    rec = json.load(open(path))
    t = bench.measured_traffic(rec["kernel"], rec["workload"])
    if rec["gemm_source_sha256"] == bench.gemm_source_sha256():
        assert t is not None and t == pytest.approx(rec["traffic_bytes_per_launch"])
    else:
        # counters taken with another GEMM source are not reported
        assert t is None
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
