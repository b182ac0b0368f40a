#!/usr/bin/env python3
"""Throughput of the finite-temperature TD-DMRG correlation loop on one GPU.

Workload: the rubrene-shaped Holstein-Peierls ring (21 molecules, 4 local
modes per molecule and 1 bond mode per bond, 10 phonon levels, purified MPS
bond dimension 128, T = 300 K), synthetic seeded parameters.

A step is one step of the C(t) loop: one second-order one-site TDVP step of
Psi_beta and one of j Psi_beta (run concurrently on two streams), and the
overlap <Psi|j|Phi>.  The inputs (Psi_beta from the imaginary-time
preparation in float64, whose one-site steps expand the bonds up to D, and
j Psi_beta compressed to D) are prepared before the timed region and stay
resident in HBM.  The headline value is the mixed-precision path (complex64 contractions
on MFMA, float64 Krylov/QR/norms).  From the same inputs the first
--compare-steps steps are then run in float64 (Krylov tolerance 1e-14), the
reference for the C(t) and window-mobility errors, and with the BF16x3
split-product contractions.  The oracle's time for a pair-step is assembled
from its kernels timed at every site shape of the two states (cpu_baseline).

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
# TFLOP/s, dense MFMA peaks of MI355X (FP32, FP64, BF16)
PEAK = {"c64": 157.3, "c128": 78.6, "bf16": 2516.6}


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


def _traffic_path(workload_name):
    return os.path.join(HERE, "profiles", f"traffic_{workload_name}.json")


def measured_traffic(kernel, workload_name):
    """HBM bytes per launch of `kernel` from the committed counter record
    (two rocprofv3 --pmc passes, FETCH_SIZE then WRITE_SIZE, calibrated by a
    copy of known size; written by --traffic), or None when the record has no
    entry for this kernel and workload or the GEMM source changed since the
    counters were taken."""
    path = _traffic_path(workload_name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("workload") != workload_name or rec.get("gemm_source_sha256") != gemm_source_sha256():
        return None
    ent = rec.get("kernels", {}).get(kernel)
    return None if ent is None else float(ent["traffic_bytes_per_launch"])


def _windows(log_path):
    """Timed-steps window (t0, t1) and calibration-copy window (t0, t1, bytes),
    boot-clock ns, as printed to `log_path` by a run of this script."""
    import re
    windows = {}
    with open(log_path) as f:
        for line in f:
            m = re.search(r"timed region boottime_ns (\d+) (\d+)", line)
            if m and "timed steps" not in windows:
                windows["timed steps"] = (int(m.group(1)), int(m.group(2)))
            m = re.search(r"calibration copy of (\d+) bytes boottime_ns (\d+) (\d+)", line)
            if m and "calibration copy" not in windows:
                windows["calibration copy"] = (int(m.group(2)), int(m.group(3)), int(m.group(1)))
    return windows


def _rows_in(csv_path, windows):
    import csv
    sel = {k: [] for k in windows}
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            st = int(row["Start_Timestamp"])
            for k, w in windows.items():
                if w[0] <= st <= w[1]:
                    sel[k].append(row)
    return sel


def summarize(kind, csv_path, log_path):
    """Summary of rocprofv3 CSV rows (kernel trace or counter collection)
    whose dispatch started inside the first timed window this script printed
    to `log_path` ("[bench] timed region boottime_ns t0 t1")."""
    windows = _windows(log_path)
    if "timed steps" not in windows:
        raise SystemExit("no timed window in the log")
    sel = _rows_in(csv_path, windows)
    for label in windows:
        summarize_rows(kind, label, windows[label][:2], sel[label])


def traffic_record(fetch_csv, fetch_log, write_csv, write_log, workload_name, commands):
    """HBM traffic per launch of every GEMM instance in the timed steps, from
    a FETCH_SIZE pass and a WRITE_SIZE pass (KiB per dispatch, counter
    collection CSVs with their logs), each scaled by what the same counter
    reads for the calibration copy of that run (a device copy of known size,
    which reads and writes its size once)."""
    import collections
    out = {"workload": workload_name, "gemm_source_sha256": gemm_source_sha256(),
           "commands": commands, "kernels": {}}
    per = collections.defaultdict(dict)
    for tag, csv_path, log_path, counter in (("fetch", fetch_csv, fetch_log, "FETCH_SIZE"),
                                             ("write", write_csv, write_log, "WRITE_SIZE")):
        windows = _windows(log_path)
        if "timed steps" not in windows or "calibration copy" not in windows:
            raise SystemExit(f"{log_path}: timed or calibration window missing")
        sel = _rows_in(csv_path, windows)
        copy_kib = sum(float(r["Counter_Value"]) for r in sel["calibration copy"]
                       if r["Counter_Name"] == counter)
        copy_bytes = windows["calibration copy"][2]
        factor = copy_bytes / 1024.0 / copy_kib
        out["calibration_copy_bytes"] = copy_bytes
        out[f"{tag}_size_kib_for_copy"] = copy_kib
        out[f"{tag}_factor"] = factor
        kib = collections.defaultdict(float)
        disp = collections.defaultdict(set)
        for r in sel["timed steps"]:
            if r["Counter_Name"] != counter or "gemm" not in r["Kernel_Name"]:
                continue
            name = r["Kernel_Name"].split("(")[0].replace("void ", "").strip()
            kib[name] += float(r["Counter_Value"])
            disp[name].add(r.get("Dispatch_Id") or len(disp[name]))
        for name in kib:
            n = len(disp[name])
            per[name][f"{tag}_size_kib_in_window"] = kib[name]
            per[name][f"{tag}_dispatches_in_window"] = n
            per[name][f"{tag}_bytes_per_launch"] = kib[name] * 1024.0 * factor / n
    for name, e in per.items():
        if "fetch_bytes_per_launch" in e and "write_bytes_per_launch" in e:
            e["traffic_bytes_per_launch"] = e["fetch_bytes_per_launch"] + e["write_bytes_per_launch"]
            out["kernels"][name] = e
    return out


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
    prec = kind >> 3
    tin = "double" if prec == 0 else "float"
    tout = "double" if (kind & 4) else tin
    ak = "true" if (kind & 2) else "false"
    bk = "true" if (kind & 1) else "false"
    if prec == 2:
        return f"ftd::gemm_bx3_kernel<{tout}, {ak}, {bk}>"
    return f"ftd::gemm_kernel<{tin}, {tout}, {ak}, {bk}>"


def workload(name):
    from paper_2003_13245_amd import workloads as W
    if name == "headline":
        return W.headline()
    if name == "small":
        return W.rubrene_shaped(n_mol=5, n_loc=2, n_nl=1, levels=6, D=32, n_imag=8)
    if name == "medium":
        return W.rubrene_shaped(n_mol=11, n_loc=4, n_nl=1, levels=10, D=64, n_imag=16)
    if name == "large":
        return W.large_rubrene_shaped()
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
    for i in range(steps):
        api.tdvp_pair(ctx, H, psi, phi, dt_real=dt, tol=tol, mmax=mmax)
        C.append(api.overlap(ctx, psi, J, phi))
        if steps >= 20 and (i + 1) % 10 == 0:
            log(f"[bench] step {i + 1}/{steps}")
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


def blas_info():
    """(threads, vendor) of the BLAS numpy uses on this host."""
    try:
        from threadpoolctl import threadpool_info
        pools = [p for p in threadpool_info() if p.get("user_api") == "blas"]
        if pools:
            return int(max(p.get("num_threads", 1) for p in pools)), pools[0].get("internal_api", "?")
    except Exception:
        pass
    return os.cpu_count() or 1, "?"


def oracle_kernel_times(wl, states, rep_s=0.25):
    """The oracle's H_eff, gauge QR, environment-update and K_eff times on
    this host at every distinct site shape of the two states, each timed once
    (repeated up to rep_s); returns ({(Dl, Dr, W shape): times}, seconds of
    CPU work spent)."""
    from oracle import mpo as OM
    from oracle import tdvp as T
    Hw = OM.hamiltonian_mpo(wl.model)
    rng = np.random.default_rng(0)
    cz = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)

    def timed(f):
        n, t0 = 0, time.perf_counter()
        while True:
            f()
            n += 1
            el = time.perf_counter() - t0
            if el > rep_s or n >= 3:
                return el / n

    cache = {}
    t_sample = time.perf_counter()
    for bonds in states:
        L = len(Hw)
        for i in range(L):
            W = Hw[i]
            d = W.shape[2]
            a = 1 if i == 0 else bonds[i - 1]
            b = 1 if i == L - 1 else bonds[i]
            key = (a, b, W.shape)
            if key in cache:
                continue
            Le, Re, A = cz(W.shape[0], a, a), cz(W.shape[1], b, b), cz(a, d, d, b)
            C, Lb = cz(b, b), cz(W.shape[1], b, b)
            t_h = timed(lambda: T.heff_apply(Le, W, Re, A))
            t_q = timed(lambda: T.qr_pos(A.reshape(a * d * d, b)))
            t_e = timed(lambda: T.left_env(Le, A, W, A))
            t_k = timed(lambda: T.keff_apply(Lb, Re, C)) if i < L - 1 else 0.0
            cache[key] = (t_h, t_q, t_e, t_k)
    return cache, time.perf_counter() - t_sample


def assemble_pair_step(wl, states, times, krylov_mean):
    """Seconds of one oracle pair-step from the kernel times: one state-step
    visits every site twice (left-to-right, right-to-left sweep); a visit is
    krylov_mean H_eff matvecs (the GPU run's mean Krylov vectors per
    exponential), one gauge QR, one environment update and krylov_mean K_eff
    matvecs on the bond; a pair-step is both states plus one overlap (one
    transfer step per site)."""
    from oracle import mpo as OM
    Hw = OM.hamiltonian_mpo(wl.model)
    t_step = 0.0
    for bonds in states:
        L = len(Hw)
        for i in range(L):
            a = 1 if i == 0 else bonds[i - 1]
            b = 1 if i == L - 1 else bonds[i]
            t_h, t_q, t_e, t_k = times[(a, b, Hw[i].shape)]
            t_step += 2 * (krylov_mean * (t_h + t_k) + t_q + t_e) + t_e / len(states)
    return t_step


def cpu_baseline(wl, states, krylov_mean, rep_s=0.25):
    """The oracle's time for one pair-step of this workload, assembled from
    the oracle's own kernels timed on this host at every distinct site shape
    of the two states as they enter the timed steps (not extrapolated from
    one shape)."""
    times, el = oracle_kernel_times(wl, states, rep_s)
    t_step = assemble_pair_step(wl, states, times, krylov_mean)
    cores, blas = blas_info()
    return {"value": 1.0 / t_step, "unit": "pair-steps/s", "cores": cores, "kind": "oracle",
            "blas": blas, "seconds_per_pair_step": t_step,
            "sample": f"oracle H_eff, K_eff, environment and QR kernels timed at each of the "
                      f"{len(times)} distinct site shapes of the two prepared states "
                      f"({el:.1f} s of CPU work), assembled into one pair-step with "
                      f"{krylov_mean:.2f} Krylov vectors per exponential (the GPU run's mean)"}


def c_err(C, ref, c0):
    """err_C = max_k |C_k - C_ref_k| / |C_ref(0)|."""
    return float(np.abs(np.asarray(C) - np.asarray(ref)).max() / abs(c0))


def mu_window(C, dt, beta, c0):
    """Kubo integral (beta / e0) int Re C dt over the timed window (trapezoid,
    C(0) = c0 first), e0 = 1."""
    c = np.concatenate([[c0], np.asarray(C)])
    return float(beta * dt * (c.real.sum() - 0.5 * (c[0].real + c[-1].real)))


def roofline_entries(st, peak_of_kind, workload_name):
    out = []
    for k in range(32):
        n = st["kind_launches"][k]
        if n == 0 or st["kind_ms"][k] <= 0:
            continue
        ach = st["kind_flops"][k] / st["kind_ms"][k] / 1e9
        peak = peak_of_kind(k)
        out.append({"kernel": kernel_name(k), "launches": n,
                    "traffic": measured_traffic(kernel_name(k), workload_name),
                    "avg_launch_ms": st["kind_ms"][k] / n,
                    "achieved": ach, "peak": peak, "frac": ach / peak,
                    "algorithmic_flops_per_launch": st["kind_flops"][k] / n,
                    "algorithmic_bytes_per_launch": st["kind_bytes"][k] / n})
    return sorted(out, key=lambda e: -e["avg_launch_ms"] * e["launches"])


def kernel_only(workload_name, n_repeat=200):
    """The H_eff matvec alone, repeated, at the workload's phonon-site shape
    (headline: D x d x d x D = 128 x 10 x 10 x 128; large: 256 x 12 x 12 x
    256) with the bulk MPO channels of the rubrene-shaped ring (a 3-molecule
    ring of the same modes has the same site), with random site and
    environment tensors, in each contraction precision: the library's device
    timing of every GEMM instance, as one JSON line."""
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_2003_13245_amd import api
    from paper_2003_13245_amd import workloads as W
    if workload_name == "large":
        wl = W.rubrene_shaped(n_mol=3, n_loc=6, n_nl=2, levels=12, D=256)
    else:
        wl = W.rubrene_shaped(n_mol=3)
    Dmax = wl.run.D
    ctx = api.Context(0)
    H, _ = api.mpo_build(ctx, wl.model)
    dims, _ = H.info()
    L = len(dims)
    site = next(i for i in range(L // 2, L) if dims[i] > 2)
    rng = np.random.default_rng(5)
    bonds = [min(Dmax, int(min(float(np.prod(dims[: i + 1].astype(float)) ** 2),
                              float(np.prod(dims[i + 1:].astype(float)) ** 2)))) for i in range(L - 1)]
    # Gaussian tensors scaled so that every transfer step keeps the
    # environments of order one (values do not change the timing, overflow
    # would only make the output unreadable)
    tensors = []
    for i in range(L):
        a, b = 1 if i == 0 else bonds[i - 1], 1 if i == L - 1 else bonds[i]
        t = W.random_site_tensor(rng, a, int(dims[i]), b)
        tensors.append(t / np.sqrt(2.0 * a * int(dims[i]) ** 2))
    x = tensors[site]
    out = {"mode": "kernel-only", "workload": workload_name, "site_shape": list(x.shape),
           "repeats": n_repeat}
    for prec, peak in (("c64", PEAK["c64"]), ("bf16x3", PEAK["bf16"]), ("c128", PEAK["c128"])):
        g = api.mps_from_host(ctx, tensors)
        g.set_precision(prec)
        api.heff_apply(ctx, H, g, site, x, n_repeat=5)
        ctx.stats_reset()
        ctx.set_timing(True)
        ctx.synchronize()
        t0 = time.perf_counter()
        api.heff_apply(ctx, H, g, site, x, n_repeat=n_repeat)
        ctx.synchronize()
        el = time.perf_counter() - t0
        st = ctx.stats()
        ctx.set_timing(False)
        res = {"wall_ms_per_matvec": el / n_repeat * 1e3,
               "heff_tflops": st["heff_flops"] / max(st["heff_ms"], 1e-9) / 1e9, "kernels": []}
        for k in range(32):
            n = st["kind_launches"][k]
            if n:
                ach = st["kind_flops"][k] / st["kind_ms"][k] / 1e9
                res["kernels"].append({"kernel": kernel_name(k), "launches": n,
                                       "avg_us": st["kind_ms"][k] / n * 1e3,
                                       "gflop_per_launch": st["kind_flops"][k] / n / 1e9,
                                       "achieved": ach, "peak": peak, "frac": ach / peak})
        out[prec] = res
        log(f"[bench] kernel-only {prec}: {res['wall_ms_per_matvec']:.3f} ms per matvec")
        del g
    out["lanczos"] = lanczos_only(api, ctx, H, tensors, site, -0.5j * wl.run.dt,
                                  max(10, n_repeat // 10))
    print(json.dumps(out), flush=True)
    ctx.close()


def lanczos_traffic(n, m):
    """Algorithmic HBM bytes of the float64 Lanczos vector kernels in one
    Krylov exponential of m vectors on n complex elements with both
    Gram-Schmidt passes (one vector pass is 16 n bytes): the projections read
    w once per eight basis vectors; the fused first correction and second
    projection, and the second correction with its norm, each read the basis
    and w and write w; the normalisation reads and writes w (not after the
    converged iteration); the final combination reads the m vectors and
    writes the result; the start reads x for its norm, copies it and scales
    the copy."""
    v = 16.0 * n
    t = {"multidot_w1_partial": 0.0, "multiaxpy_dot_partial": 0.0,
         "multiaxpy_nrm_partial": 0.0, "lanczos_post_kernel": 0.0,
         "lincomb_kernel": (m + 1) * v, "nrm2_partial+copy_kernel+scale_dev_kernel": 5 * v}
    for k in range(m):
        j = k + 1
        t["multidot_w1_partial"] += (j - (-j // 8)) * v
        t["multiaxpy_dot_partial"] += (j + 2) * v
        t["multiaxpy_nrm_partial"] += (j + 2) * v
        if k < m - 1:
            t["lanczos_post_kernel"] += 2 * v
    return t


def lanczos_only(api, ctx, H, tensors, site, z, n_exp):
    """The Krylov exponential exp(z H_eff) x at one site (float64
    contractions, Krylov tolerance 1e-14, so that both Gram-Schmidt passes
    always run and every launch's traffic is known), repeated: its Krylov
    count, wall time per exponential and the algorithmic bytes of each Lanczos
    kernel per exponential.  Divided by the kernels' total times in a kernel
    trace of the same command (over all 2 + n_exp exponentials it runs) they
    give the achieved bandwidth."""
    g = api.mps_from_host(ctx, tensors)
    g.set_precision("c128")
    x = tensors[site]
    try:
        api.heff_expm(ctx, H, g, site, x, z)   # warm-up: environments, buffers
        ctx.synchronize()
        t0 = time.perf_counter()
        _, m1 = api.heff_expm(ctx, H, g, site, x, z)
        ctx.synchronize()
        t1 = time.perf_counter()
        _, m = api.heff_expm(ctx, H, g, site, x, z, n_repeat=n_exp)
        ctx.synchronize()
        t2 = time.perf_counter()
    except api.FtdError as e:
        return {"error": str(e)}
    finally:
        del g
    # both calls build the same environments: their difference is n_exp - 1
    # exponentials
    per = ((t2 - t1) - (t1 - t0)) / (n_exp - 1)
    n = int(np.prod(x.shape))
    traffic = lanczos_traffic(n, m)
    res = {"precision": "c128", "z": [z.real, z.imag], "krylov_vectors": m,
           "krylov_vectors_first": m1, "exponentials_total": 2 + n_exp,
           "wall_ms_per_exp": per * 1e3, "vector_bytes": 16 * n,
           "bytes_per_exp": traffic,
           "lanczos_bytes_per_exp": sum(traffic.values())}
    log(f"[bench] kernel-only Lanczos: m = {m}, {per * 1e3:.3f} ms per exponential, "
        f"{res['lanczos_bytes_per_exp'] / 1e9:.2f} GB of vector traffic")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="headline")
    ap.add_argument("--compare-steps", type=int, default=10,
                    help="steps of the bf16x3 and float64 comparison runs (at most --steps)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64 comparison run")
    ap.add_argument("--no-bf16x3", action="store_true", help="skip the bf16x3 run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n-grow", type=int, default=None,
                    help="growth steps of the preparation (default: the workload's; <0 adaptive)")
    ap.add_argument("--expand-tol", type=float, default=None,
                    help="bond expansion threshold of the preparation's TDVP steps "
                         "(default: the workload's; 0 turns expansion off)")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="after timing, copy this many MiB device-to-device inside its own "
                         "profiler region (HBM counter calibration)")
    ap.add_argument("--verbose", type=int, default=1,
                    help="library progress lines on stderr (0 silent, 2 per compression)")
    ap.add_argument("--state-cache", default=None, metavar="DIR",
                    help="load Psi_beta and j Psi_beta of this workload from DIR when a "
                         "previous run saved them there, else prepare them and save them "
                         "(lets profiled runs skip the preparation)")
    ap.add_argument("--krylov-tol", type=float, default=None,
                    help="Lanczos stop tolerance of the mixed runs (default: the workload's)")
    ap.add_argument("--summarize", nargs=3, metavar=("KIND", "CSV", "LOG"),
                    help="summarise rocprofv3 CSV rows (KIND trace or pmc) of the timed window "
                         "recorded in LOG, then exit (no GPU)")
    ap.add_argument("--traffic", nargs=4,
                    metavar=("FETCH_CSV", "FETCH_LOG", "WRITE_CSV", "WRITE_LOG"),
                    help="write profiles/traffic_<workload>.json from a FETCH_SIZE and a "
                         "WRITE_SIZE counter pass of this script (run with "
                         "--calibration-copy-mib), then exit (no GPU)")
    ap.add_argument("--kernel-only", action="store_true",
                    help="time the H_eff contraction kernels alone at the phonon-site "
                         "shape of --workload (large: 256x12x12x256, otherwise the "
                         "headline's 128x10x10x128) in every precision (one JSON line), "
                         "then exit")
    ap.add_argument("--traffic-commands", nargs="*", default=[],
                    help="the commands of the two counter passes, recorded with --traffic")
    args = ap.parse_args()
    if args.summarize:
        summarize(*args.summarize)
        return
    if args.traffic:
        rec = traffic_record(*args.traffic, workload(args.workload).name, args.traffic_commands)
        with open(_traffic_path(rec["workload"]), "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps({k: v["traffic_bytes_per_launch"] for k, v in rec["kernels"].items()}))
        return
    if args.kernel_only:
        kernel_only(args.workload, n_repeat=200 if args.workload != "large" else 30)
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
    if args.expand_tol is not None:
        r.expand_tol = args.expand_tol
    ctx = api.Context(0)
    ctx.set_verbose(args.verbose)
    H, J = api.mpo_build(ctx, m)
    tol = args.krylov_tol if args.krylov_tol is not None else r.krylov_tol
    mmax = r.krylov_mmax

    cache, cached = None, False
    if args.state_cache:
        os.makedirs(args.state_cache, exist_ok=True)
        cache = {k: os.path.join(args.state_cache, f"{wl.name}_{k}")
                 for k in ("psi.ftd", "phi.ftd", "meta.json")}
    if cache and os.path.exists(cache["meta.json"]):
        with open(cache["meta.json"]) as f:
            meta = json.load(f)
        psi_beta = api.mps_load(ctx, cache["psi.ftd"])
        phi0 = api.mps_load(ctx, cache["phi.ftd"])
        logz, t_prep, t_j = meta["ln_Z"], meta["prep_s"], meta["jcompress_s"]
        cached = True
        log(f"[bench] Psi_beta and j|Psi> loaded from {args.state_cache} (prepared in "
            f"{t_prep:.1f} s + {t_j:.1f} s by an earlier run)")
    else:
        log(f"[bench] {wl.name}: preparing Psi_beta ({r.n_imag} imaginary steps, D={r.D}, "
            f"{r.prep_precision} contractions, Krylov tol {r.prep_krylov_tol:g}, "
            f"expansion {r.expand_tol:g})")
        t0 = time.perf_counter()
        psi_beta, logz = api.thermal_prep(ctx, H, r.beta, r.n_imag, r.n_grow, r.D,
                                          cutoff=r.cutoff, precision=r.prep_precision,
                                          tol=r.prep_krylov_tol, mmax=mmax,
                                          expand_tol=r.expand_tol)
        t_prep = time.perf_counter() - t0
        t0 = time.perf_counter()
        phi0 = api.apply_compress(ctx, J, psi_beta, r.D, r.cutoff)
        t_j = time.perf_counter() - t0
        if cache:
            psi_beta.save(cache["psi.ftd"])
            phi0.save(cache["phi.ftd"])
            with open(cache["meta.json"], "w") as f:
                json.dump({"ln_Z": logz, "prep_s": t_prep, "jcompress_s": t_j}, f)
    bonds = psi_beta.info()["bond_dims"]
    log(f"[bench] prep {t_prep:.1f} s, ln Z = {logz:.6f}, bonds max {max(bonds)} "
        f"mean {sum(bonds) / len(bonds):.1f}")
    pbonds = phi0.info()["bond_dims"]
    log(f"[bench] j|Psi> compressed in {t_j:.1f} s, bonds max {max(pbonds)} "
        f"mean {sum(pbonds) / len(pbonds):.1f}")
    c0 = api.overlap(ctx, psi_beta, J, phi0)
    # the timed steps run in the workload's precision from the float64 inputs
    psi0 = _as(api, ctx, psi_beta, wl.precision)
    phi0 = _as(api, ctx, phi0, wl.precision)

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
        c0t = time.clock_gettime_ns(time.CLOCK_BOOTTIME)
        dst.copy_(src)
        torch.cuda.synchronize()
        c1t = time.clock_gettime_ns(time.CLOCK_BOOTTIME)
        roctx.pause()
        log(f"[bench] calibration copy of {n * 4} bytes boottime_ns {c0t} {c1t}")
        del src, dst
    sps = args.steps / el_mix
    log(f"[bench] mixed: {el_mix / args.steps * 1e3:.1f} ms/step, H_eff "
        f"{st['heff_flops'] / max(st['heff_ms'], 1e-9) / 1e9:.1f} TFLOP/s")

    peak_of_kind = lambda k: {0: PEAK["c128"], 1: PEAK["c64"], 2: PEAK["bf16"]}[k >> 3]
    out = {
        "metric": METRIC, "value": sps, "unit": "pair-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el_mix / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": wl.precision, "data": "synthetic",
        "config": {"workload": wl.name, "n_mol": m.n_mol, "local_modes": m.n_loc,
                   "bond_modes": m.n_nl, "levels": m.levels_loc, "D": r.D,
                   "T_K": r.T_K, "dt_fs": r.dt_fs, "krylov_tol": tol, "n_imag": r.n_imag,
                   "n_grow": r.n_grow, "expand_tol": r.expand_tol,
                   "prep_precision": r.prep_precision, "prep_krylov_tol": r.prep_krylov_tol,
                   "psi_bond_max": max(bonds),
                   "psi_bond_mean": round(sum(bonds) / len(bonds), 1),
                   "phi_bond_max": max(pbonds), "phi_bond_mean": round(sum(pbonds) / len(pbonds), 1)},
        "heff_tflops": st["heff_flops"] / max(st["heff_ms"], 1e-9) / 1e9,
        "whole_step_tflops": st["all_flops"] / el_mix / 1e12,
        "matvecs_per_step": st["matvecs"] / args.steps,
        "krylov_mean": st["krylov_vectors"] / max(st["expm_calls"], 1),
        "prep_s": t_prep, "jcompress_s": t_j, "ln_Z": logz, "state_from_cache": cached,
    }
    dom = st["dom_kind"]
    dom_avg_ms = st["dom_ms"] / max(st["dom_launches"], 1)
    achieved = st["dom_flops"] / max(st["dom_ms"], 1e-12) / 1e9     # TFLOP/s
    peak = peak_of_kind(dom)
    out["roofline"] = {"bound": "mfma", "achieved": achieved, "peak": peak,
                       "unit": "TFLOP/s", "frac": achieved / peak,
                       "traffic": measured_traffic(kernel_name(dom), wl.name),
                       "kernel": kernel_name(dom),
                       "avg_launch_ms": dom_avg_ms, "launches": st["dom_launches"],
                       "algorithmic_bytes_per_launch":
                           st["dom_bytes"] / max(st["dom_launches"], 1),
                       "algorithmic_flops_per_launch":
                           st["dom_flops"] / max(st["dom_launches"], 1),
                       "mfma_executed_frac": achieved / peak * (0.75 if dom >> 3 == 1 else 1.0)}
    out["roofline_all"] = roofline_entries(st, peak_of_kind, wl.name)
    ncmp = max(1, min(args.compare_steps, args.steps))
    refs = {}
    if not args.no_fp64:
        C64, el64, st64 = run_steps(api, ctx, H, J, _as(api, ctx, psi0, "c128"),
                                    _as(api, ctx, phi0, "c128"), ncmp, r.dt, 1e-14, mmax, True)
        refs["c128"] = C64
        out["fp64_steps_per_s"] = ncmp / el64
        out["speedup_vs_fp64"] = sps / out["fp64_steps_per_s"]
        out["fp64_heff_tflops"] = st64["heff_flops"] / max(st64["heff_ms"], 1e-9) / 1e9
        out["c_rel_err_vs_fp64"] = c_err(C_mix[:ncmp], C64, c0)
        mu64 = mu_window(C64, r.dt, r.beta, c0)
        out["mu_rel_err_vs_fp64"] = abs(mu_window(C_mix[:ncmp], r.dt, r.beta, c0) - mu64) / abs(mu64)
        out["compare_steps"] = ncmp
        log(f"[bench] fp64 (Krylov tol 1e-14): {el64 / ncmp * 1e3:.1f} ms/step; C(t) rel err "
            f"{out['c_rel_err_vs_fp64']:.2e} over {ncmp} steps")
    if not args.no_bf16x3:
        Cb, elb, stb = run_steps(api, ctx, H, J, _as(api, ctx, psi0, "bf16x3"),
                                 _as(api, ctx, phi0, "bf16x3"), ncmp, r.dt, tol, mmax, True)
        bx = {"steps_per_s": ncmp / elb, "ms_per_step": elb / ncmp * 1e3,
              "heff_tflops": stb["heff_flops"] / max(stb["heff_ms"], 1e-9) / 1e9,
              "whole_step_tflops": stb["all_flops"] / elb / 1e12,
              "roofline_all": roofline_entries(stb, peak_of_kind, wl.name)}
        if "c128" in refs:
            bx["c_rel_err_vs_fp64"] = c_err(Cb, refs["c128"], c0)
            mu64 = mu_window(refs["c128"], r.dt, r.beta, c0)
            bx["mu_rel_err_vs_fp64"] = abs(mu_window(Cb, r.dt, r.beta, c0) - mu64) / abs(mu64)
            bx["speedup_vs_fp64"] = bx["steps_per_s"] / out["fp64_steps_per_s"]
        out["bf16x3"] = bx
        log(f"[bench] bf16x3: {bx['ms_per_step']:.1f} ms/step")
    if not args.no_cpu_baseline:
        states = [bonds, pbonds]
        out["cpu_baseline"] = cpu_baseline(wl, states, out["krylov_mean"])
    ctx.synchronize()
    print(json.dumps(out), flush=True)
    # release every device handle and the context before interpreter exit
    del psi_beta, phi0, psi0, H, J
    ctx.close()


def _as(api, ctx, psi, precision):
    """A copy of psi whose contractions run in `precision`."""
    c = psi.copy()
    c.set_precision(precision)
    return c


if __name__ == "__main__":
    main()
