#!/usr/bin/env python3
"""Throughput of the finite-temperature TD-DMRG correlation loop on one GPU.

Workload: the rubrene-shaped Holstein-Peierls ring (21 molecules, 4 local
modes per molecule and 1 bond mode per bond, 10 phonon levels, purified MPS
bond dimension 128, T = 300 K), synthetic seeded parameters.

A step is one step of the C(t) loop: one second-order one-site TDVP step of
Psi_beta and one of j Psi_beta (run concurrently on two streams), and the
overlap <Psi|j|Phi>.  The inputs
(Psi_beta from the imaginary-time preparation and j Psi_beta compressed to
D) are prepared before the timed region and stay resident in HBM.  The
headline value is the mixed-precision path (complex64 contractions on MFMA,
float64 Krylov/QR/norms); the same steps are then repeated in float64 from
the same inputs, which gives the speedup and the C(t) error of the mixed path.

Prints one JSON line.  `--gpus N` with N > 1 exits: this build targets one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "TDVP steps/s + H_eff TFLOP/s, mixed vs FP64 at C(t) rel err 1e-4, D=128"
PEAK = {"c64": 157.3, "c128": 78.6}   # TFLOP/s, dense MFMA (FP32, FP64)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Roctx:
    """roctx profiler pause/resume: with `rocprofv3 --selected-regions` only
    the bracketed regions (the timed steps) are traced.  No-op without the
    library or without a profiler."""

    def __init__(self):
        import ctypes
        self.lib = None
        for path in ("/opt/rocm/lib/librocprofiler-sdk-roctx.so", "librocprofiler-sdk-roctx.so"):
            try:
                lib = ctypes.CDLL(path)
            except OSError:
                continue
            if hasattr(lib, "roctxProfilerResume") and hasattr(lib, "roctxProfilerPause"):
                for f in (lib.roctxProfilerResume, lib.roctxProfilerPause):
                    f.argtypes = [ctypes.c_uint64]   # roctx_thread_id_t, 0 = whole process
                    f.restype = ctypes.c_int
                self.lib = lib
                break

    def resume(self):
        if self.lib is not None:
            self.lib.roctxProfilerResume(0)

    def pause(self):
        if self.lib is not None:
            self.lib.roctxProfilerPause(0)


def gemm_source_sha256():
    import hashlib
    path = os.path.join(HERE, "paper_2003_13245_amd", "csrc", "gemm.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel, workload_name):
    """HBM bytes per launch of `kernel` from the committed counter record
    (two rocprofv3 --pmc passes, FETCH_SIZE then WRITE_SIZE, calibrated by a
    copy of known size), or None when there is none for this kernel and
    workload or the kernel source changed since it was taken."""
    path = os.path.join(HERE, "profiles", f"traffic_{workload_name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel") != kernel or rec.get("gemm_source_sha256") != gemm_source_sha256():
        return None
    return float(rec["traffic_bytes_per_launch"])


def summarize(kind, csv_path, log_path):
    """Summary of rocprofv3 CSV rows (kernel trace or counter collection)
    whose dispatch started inside the first timed window this script printed
    to `log_path` ("[bench] timed region boottime_ns t0 t1")."""
    import collections
    import csv
    import re
    windows = {}
    with open(log_path) as f:
        for line in f:
            for label, pat in (("timed steps", r"timed region boottime_ns (\d+) (\d+)"),
                               ("calibration copy",
                                r"calibration copy of \d+ bytes boottime_ns (\d+) (\d+)")):
                m = re.search(pat, line)
                if m and label not in windows:
                    windows[label] = (int(m.group(1)), int(m.group(2)))
    if "timed steps" not in windows:
        raise SystemExit("no timed window in the log")
    sel = {k: [] for k in windows}
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            st = int(row["Start_Timestamp"])
            for k, (a, b) in windows.items():
                if a <= st <= b:
                    sel[k].append(row)
    for label in windows:
        summarize_rows(kind, label, windows[label], sel[label])


def summarize_rows(kind, label, window, rows):
    import collections
    t0, t1 = window
    out = [f"[{label}] window {(t1 - t0) / 1e9:.3f} s, dispatches in window {len(rows)}"]
    if kind == "trace":
        acc = collections.defaultdict(lambda: [0, 0, 0, 1 << 62])
        for row in rows:
            d = int(row["End_Timestamp"]) - int(row["Start_Timestamp"])
            a = acc[row["Kernel_Name"]]
            a[0] += 1
            a[1] += d
            a[2] = max(a[2], d)
            a[3] = min(a[3], d)
        tot = sum(a[1] for a in acc.values())
        out.append(f"kernel time in window {tot / 1e6:.1f} ms (summed over both streams)")
        out.append("calls\ttotal_ms\tavg_us\tmin_us\tmax_us\tshare\tkernel")
        for name, (n, t, mx, mn) in sorted(acc.items(), key=lambda kv: -kv[1][1])[:30]:
            out.append(f"{n}\t{t / 1e6:.2f}\t{t / n / 1e3:.2f}\t{mn / 1e3:.2f}\t{mx / 1e3:.2f}\t"
                       f"{100 * t / tot:.1f}%\t{name[:100]}")
    else:
        acc = collections.defaultdict(list)
        for row in rows:
            acc[(row["Kernel_Name"], row["Counter_Name"])].append(float(row["Counter_Value"]))
        out.append("counter\tdispatches\tsum_KiB\tmax_KiB\tkernel")
        for (name, cn), v in sorted(acc.items(), key=lambda kv: -sum(kv[1])):
            out.append(f"{cn}\t{len(v)}\t{sum(v):.6g}\t{max(v):.6g}\t{name[:100]}")
    print("\n".join(out))


def kernel_name(kind):
    """Name of the GEMM kernel instance with identity `kind` (see ftd_stats)."""
    tin = "double" if (kind >> 3) == 0 else "float"
    tout = "double" if (kind & 4) else tin
    ak = "true" if (kind & 2) else "false"
    bk = "true" if (kind & 1) else "false"
    return f"ftd::gemm_kernel<{tin}, {tout}, {ak}, {bk}>"


def workload(name):
    from paper_2003_13245_amd import workloads as W
    if name == "headline":
        return W.headline()
    if name == "small":
        return W.rubrene_shaped(n_mol=5, n_loc=2, n_nl=1, levels=6, D=32, n_imag=8)
    if name == "medium":
        return W.rubrene_shaped(n_mol=11, n_loc=4, n_nl=1, levels=10, D=64, n_imag=16)
    raise SystemExit(f"unknown workload {name}")


def run_steps(api, ctx, H, J, psi0, phi0, steps, dt, tol, mmax, timing, roctx=None):
    psi, phi = psi0.copy(), phi0.copy()
    C = []
    ctx.stats_reset()
    ctx.set_timing(timing)
    ctx.synchronize()
    if roctx:
        roctx.resume()
    b0 = time.clock_gettime_ns(time.CLOCK_BOOTTIME)
    t0 = time.perf_counter()
    for _ in range(steps):
        api.tdvp_pair(ctx, H, psi, phi, dt_real=dt, tol=tol, mmax=mmax)
        C.append(api.overlap(ctx, psi, J, phi))
    ctx.synchronize()
    t1 = time.perf_counter()
    b1 = time.clock_gettime_ns(time.CLOCK_BOOTTIME)
    if roctx:
        roctx.pause()
    if timing:
        # profiler timestamps of this window select the timed dispatches
        log(f"[bench] timed region boottime_ns {b0} {b1}")
    st = ctx.stats()
    ctx.set_timing(False)
    return np.array(C), t1 - t0, st


def cpu_baseline(wl, matvecs_per_step, budget_s=20.0):
    """Oracle H_eff matvecs at the workload's widest phonon-site shape (random
    environments of the oracle MPO's channel count), scaled to a step by the
    number of matvecs one step issued on the GPU."""
    from oracle import mpo as OM
    from oracle import tdvp as T
    m = wl.model
    Hw = OM.hamiltonian_mpo(m)
    D = wl.run.D
    L = len(Hw)
    site = next(i for i in range(L // 2, L) if Hw[i].shape[2] > 2)
    W = Hw[site]
    d = W.shape[2]
    rng = np.random.default_rng(0)
    Lenv = rng.standard_normal((W.shape[0], D, D)) + 1j * rng.standard_normal((W.shape[0], D, D))
    Renv = rng.standard_normal((W.shape[1], D, D)) + 1j * rng.standard_normal((W.shape[1], D, D))
    A = rng.standard_normal((D, d, d, D)) + 1j * rng.standard_normal((D, d, d, D))
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    n, t0 = 0, time.perf_counter()
    while True:
        T.heff_apply(Lenv, W, Renv, A)
        n += 1
        el = time.perf_counter() - t0
        if el > budget_s or n >= 50:
            break
    per = el / n
    step_s = per * matvecs_per_step
    return {"value": 1.0 / step_s, "unit": "pair-steps/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{n} oracle H_eff matvecs at the D={D}, d={d} phonon-site shape "
                      f"({per:.3f} s each, {el:.1f} s total), scaled by the "
                      f"{matvecs_per_step:.0f} matvecs of one GPU step"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="headline")
    ap.add_argument("--precision", default="c64", choices=["c64", "c128"],
                    help="contraction precision of the timed steps (c128: the FP64 path)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n-grow", type=int, default=None,
                    help="growth steps of the preparation (default: the workload's; <0 adaptive)")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="after timing, copy this many MiB device-to-device inside its own "
                         "profiler region (HBM counter calibration)")
    ap.add_argument("--verbose", type=int, default=1,
                    help="library progress lines on stderr (0 silent, 2 per compression)")
    ap.add_argument("--expand-tol", type=float, default=None,
                    help="bond expansion threshold of the preparation's TDVP steps "
                         "(default: the workload's; 0 turns expansion off)")
    ap.add_argument("--krylov-tol", type=float, default=None,
                    help="Lanczos stop tolerance (default: the workload's)")
    ap.add_argument("--summarize", nargs=3, metavar=("KIND", "CSV", "LOG"),
                    help="summarise rocprofv3 CSV rows (KIND trace or pmc) of the timed window "
                         "recorded in LOG, then exit (no GPU)")
    args = ap.parse_args()
    if args.summarize:
        summarize(*args.summarize)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_2003_13245_amd import api

    wl = workload(args.workload)
    m, r = wl.model, wl.run
    if args.n_grow is not None:
        r.n_grow = args.n_grow
    ctx = api.Context(0)
    ctx.set_verbose(args.verbose)
    H, J = api.mpo_build(ctx, m)
    tol = args.krylov_tol if args.krylov_tol is not None else r.krylov_tol
    mmax = r.krylov_mmax

    log(f"[bench] {wl.name}: preparing Psi_beta ({r.n_imag} imaginary steps, D={r.D})")
    t0 = time.perf_counter()
    if args.expand_tol is not None:
        r.expand_tol = args.expand_tol
    psi_beta, logz = api.thermal_prep(ctx, H, r.beta, r.n_imag, r.n_grow, r.D, cutoff=r.cutoff,
                                      precision=args.precision, tol=tol, mmax=mmax,
                                      expand_tol=r.expand_tol)
    t_prep = time.perf_counter() - t0
    bonds = psi_beta.info()["bond_dims"]
    log(f"[bench] prep {t_prep:.1f} s, ln Z = {logz:.6f}, bonds max {max(bonds)} "
        f"mean {sum(bonds) / len(bonds):.1f}")
    t0 = time.perf_counter()
    phi0 = api.apply_compress(ctx, J, psi_beta, r.D, r.cutoff)
    t_j = time.perf_counter() - t0
    pbonds = phi0.info()["bond_dims"]
    log(f"[bench] j|Psi> compressed in {t_j:.1f} s, bonds max {max(pbonds)} "
        f"mean {sum(pbonds) / len(pbonds):.1f}")
    psi0 = psi_beta

    # warmup (untimed), then the timed mixed-precision steps
    if args.warmup:
        run_steps(api, ctx, H, J, psi0, phi0, args.warmup, r.dt, tol, mmax, False)
    roctx = Roctx()
    C_mix, el_mix, st = run_steps(api, ctx, H, J, psi0, phi0, args.steps, r.dt, tol, mmax, True,
                                  roctx)
    if args.calibration_copy_mib > 0:
        n = args.calibration_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        roctx.resume()
        c0 = time.clock_gettime_ns(time.CLOCK_BOOTTIME)
        dst.copy_(src)
        torch.cuda.synchronize()
        c1 = time.clock_gettime_ns(time.CLOCK_BOOTTIME)
        roctx.pause()
        log(f"[bench] calibration copy of {n * 4} bytes boottime_ns {c0} {c1}")
        del src, dst
    sps = args.steps / el_mix
    log(f"[bench] mixed: {el_mix / args.steps * 1e3:.1f} ms/step, H_eff "
        f"{st['heff_flops'] / max(st['heff_ms'], 1e-9) / 1e9:.1f} TFLOP/s")

    out = {
        "metric": METRIC, "value": sps, "unit": "pair-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el_mix / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic",
        "config": {"workload": wl.name, "n_mol": m.n_mol, "local_modes": m.n_loc,
                   "bond_modes": m.n_nl, "levels": m.levels_loc, "D": r.D,
                   "T_K": 300.0, "dt_fs": 0.5, "krylov_tol": tol, "n_imag": r.n_imag,
                   "n_grow": r.n_grow, "psi_bond_max": max(bonds),
                   "psi_bond_mean": round(sum(bonds) / len(bonds), 1),
                   "phi_bond_max": max(pbonds), "phi_bond_mean": round(sum(pbonds) / len(pbonds), 1)},
        "heff_tflops": st["heff_flops"] / max(st["heff_ms"], 1e-9) / 1e9,
        "matvecs_per_step": st["matvecs"] / args.steps,
        "krylov_mean": st["krylov_vectors"] / max(st["expm_calls"], 1),
        "prep_s": t_prep, "jcompress_s": t_j,
    }
    dom_avg_ms = st["dom_ms"] / max(st["dom_launches"], 1)
    achieved = st["dom_flops"] / max(st["dom_ms"], 1e-12) / 1e9     # TFLOP/s
    out["roofline"] = {"bound": "mfma", "achieved": achieved, "peak": PEAK[args.precision],
                       "unit": "TFLOP/s", "frac": achieved / PEAK[args.precision],
                       "traffic": measured_traffic(kernel_name(st["dom_kind"]), wl.name),
                       "kernel": kernel_name(st["dom_kind"]),
                       "avg_launch_ms": dom_avg_ms, "launches": st["dom_launches"],
                       "algorithmic_bytes_per_launch":
                           st["dom_bytes"] / max(st["dom_launches"], 1),
                       "algorithmic_flops_per_launch":
                           st["dom_flops"] / max(st["dom_launches"], 1)}
    if not args.no_fp64:
        C64, el64, st64 = run_steps(api, ctx, H, J, _as(api, ctx, psi0, "c128"),
                                    _as(api, ctx, phi0, "c128"), args.steps, r.dt, 1e-12,
                                    mmax, True)
        out["fp64_steps_per_s"] = args.steps / el64
        out["speedup_vs_fp64"] = sps / out["fp64_steps_per_s"]
        out["fp64_heff_tflops"] = st64["heff_flops"] / max(st64["heff_ms"], 1e-9) / 1e9
        out["c_rel_err_vs_fp64"] = float(np.abs(C_mix - C64).max() /
                                         abs(api.overlap(ctx, psi0, J, phi0)))
        log(f"[bench] fp64: {el64 / args.steps * 1e3:.1f} ms/step; C(t) rel err "
            f"{out['c_rel_err_vs_fp64']:.2e}")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, out["matvecs_per_step"])
    print(json.dumps(out), flush=True)


def _as(api, ctx, psi, precision):
    """A copy of psi whose contractions run in `precision`."""
    c = psi.copy()
    c.set_precision(precision)
    return c


if __name__ == "__main__":
    main()
