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
    out = bench.roofline_entries(st, lambda k: 157.3, "no counter record")
    assert [e["kernel"] for e in out] == ["ftd::gemm_kernel<float, double, false, true>",
                                          "ftd::gemm_kernel<float, float, true, false>"]
    assert out[0]["achieved"] == pytest.approx(75.0) and out[0]["avg_launch_ms"] == 0.2
    assert out[1]["frac"] == pytest.approx(50.0 / 157.3)
    assert out[0]["traffic"] is None


def test_cpu_baseline_assembles_a_step(bench):
    """Every distinct site shape is timed once and the step is the sum over
    both states' sites: going from 4 to 8 Krylov vectors per exponential adds
    exactly 4 x 2 (H_eff + K_eff) per site visit to the same kernel times."""
    from paper_2003_13245_amd import workloads as W
    from oracle import model as Mdl
    from oracle import mpo as OM
    wl = W.rubrene_shaped(n_mol=3, n_loc=1, n_nl=1, levels=3, D=6)
    Hw = OM.hamiltonian_mpo(wl.model)
    L = len(Mdl.site_dims(wl.model))
    bonds = [min(6, 4 ** (i + 1), 4 ** (L - 1 - i)) for i in range(L - 1)]
    states = [bonds, bonds]
    times, _ = bench.oracle_kernel_times(wl, states, rep_s=0.01)
    keys = [(1 if i == 0 else bonds[i - 1], 1 if i == L - 1 else bonds[i], Hw[i].shape)
            for i in range(L)]
    assert set(keys) == set(times)
    a = bench.assemble_pair_step(wl, states, times, 4.0)
    b = bench.assemble_pair_step(wl, states, times, 8.0)
    per_vector = sum(2 * (times[k][0] + times[k][3]) for k in keys) * len(states)
    assert b - a == pytest.approx(4.0 * per_vector, rel=1e-12)
    r = bench.cpu_baseline(wl, states, 4.0, rep_s=0.01)
    assert r["kind"] == "oracle" and r["unit"] == "pair-steps/s" and r["cores"] >= 1
    assert r["value"] > 0 and r["seconds_per_pair_step"] > 0


def test_traffic_record_matches_current_source(bench):
    """The committed counter record: its arithmetic, and that it is reported
    only for the GEMM source and workload it was taken with."""
    path = os.path.join(ROOT, "profiles", "traffic_hp_n21_loc4_nl1_d10_D128_T300.json")
    if not os.path.exists(path):
        pytest.skip("no committed counter record")
    rec = json.load(open(path))
    assert rec["kernels"], "record without kernels"
    copy_kib = rec["calibration_copy_bytes"] / 1024
    assert rec["fetch_factor"] == pytest.approx(copy_kib / rec["fetch_size_kib_for_copy"])
    assert rec["write_factor"] == pytest.approx(copy_kib / rec["write_size_kib_for_copy"])
    same = rec["gemm_source_sha256"] == bench.gemm_source_sha256()
    for name, e in rec["kernels"].items():
        fb = e["fetch_size_kib_in_window"] * 1024 * rec["fetch_factor"] / e["fetch_dispatches_in_window"]
        wb = e["write_size_kib_in_window"] * 1024 * rec["write_factor"] / e["write_dispatches_in_window"]
        assert fb + wb == pytest.approx(e["traffic_bytes_per_launch"], rel=1e-12)
        t = bench.measured_traffic(name, rec["workload"])
        # counters taken with another GEMM source are not reported
        assert (t == pytest.approx(e["traffic_bytes_per_launch"])) if same else t is None
    assert bench.measured_traffic("some other kernel", rec["workload"]) is None
    assert bench.measured_traffic(next(iter(rec["kernels"])), "another workload") is None


def test_traffic_record_from_counter_passes(bench, tmp_path):
    """--traffic: per-launch bytes = counter KiB in the timed window x 1024 x
    (copy bytes / counter KiB of the calibration copy) / dispatches."""
    ms = 1000000
    cols = "Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value,Start_Timestamp\n"
    gemm = "void ftd::gemm_kernel<float, double, true, true>(float const*, float const*)"
    for tag, counter, per_launch, copy_kib in (("f", "FETCH_SIZE", 300.0, 2048.0),
                                               ("w", "WRITE_SIZE", 100.0, 1024.0)):
        (tmp_path / f"{tag}.log").write_text(
            f"[bench] timed region boottime_ns {100 * ms} {200 * ms}\n"
            f"[bench] calibration copy of 1048576 bytes boottime_ns {300 * ms} {310 * ms}\n")
        rows = [f'1,"{gemm}",{counter},{per_launch},{120 * ms}',
                f'2,"{gemm}",{counter},{per_launch},{150 * ms}',
                f'3,"{gemm}",{counter},{per_launch},{250 * ms}',       # outside the window
                f'4,"copy_kernel(float*)",{counter},{copy_kib},{305 * ms}']
        (tmp_path / f"{tag}.csv").write_text(cols + "\n".join(rows) + "\n")
    rec = bench.traffic_record(str(tmp_path / "f.csv"), str(tmp_path / "f.log"),
                               str(tmp_path / "w.csv"), str(tmp_path / "w.log"), "wl", ["cmd"])
    e = rec["kernels"]["ftd::gemm_kernel<float, double, true, true>"]
    assert e["fetch_dispatches_in_window"] == 2 and e["write_dispatches_in_window"] == 2
    # fetch: copy of 1 MiB read as 2048 KiB -> factor 0.5; write: factor 1
    assert e["fetch_bytes_per_launch"] == pytest.approx(300.0 * 1024 * 0.5)
    assert e["write_bytes_per_launch"] == pytest.approx(100.0 * 1024)
    assert e["traffic_bytes_per_launch"] == pytest.approx(300.0 * 512 + 100.0 * 1024)


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


def test_lanczos_traffic_counts_vector_passes():
    """One Krylov vector: projection 2 passes, fused correction 3, second
    correction 3, no normalisation (the iteration converges), final
    combination 2, start 5: 15 passes of 16 n bytes; each further vector j
    adds j + ceil(j / 8) + 2 (j + 2) + 2 passes and one more for the final
    combination."""
    import bench
    n = 1000
    one = bench.lanczos_traffic(n, 1)
    assert sum(one.values()) == 15 * 16 * n
    for m in range(2, 20):
        d = sum(bench.lanczos_traffic(n, m).values()) - sum(bench.lanczos_traffic(n, m - 1).values())
        assert d == (m + -(-m // 8) + 2 * (m + 2) + 2 + 1) * 16 * n, m
