#!/usr/bin/env python3
"""Throughput of the blocked Jacobi sweep (multi-threaded wavefront diamond
blocking) on one MI355X, printed as one JSON line.

A step is one whole run of the hot path on the workload: girih_run of T
Jacobi steps of the 7-point constant-coefficient stencil on a 512^3 FP64 grid
(T = 64; every diamond row of the schedule, their prologue loads, wavefront
loops and epilogue stores).  Inputs are seeded synthetic fields already
resident in HBM; the timed region holds exactly --steps runs, bracketed by
device synchronisation.

Beside the headline value the line carries:
  roofline      the dominant kernel (the diamond-row kernel) against HBM
                peak: algorithmic bytes per launch (the paper's blocked code
                balance B_C of the plan, bytes per lattice update, times the
                updates of one launch) divided by its average launch duration,
                measured with HIP events on the launch stream inside the timed
                runs; the redundant x-halo reads of the x-chunking are reported
                apart (x_halo_read_factor), and traffic comes from the committed
                rocprofv3 counter summary when it was taken on the current
                kernel source, else null;
  cpu_baseline  the FP64 CPU oracle on the same workload, a bounded number of
                steps, on the host's cores (and on one thread), with the host's
                CPU model, sockets, memory and compiler; and the oracle on the
                other workloads for a few seconds each;
  compare       naive GPU sweep (FP64), blocked FP32 run and its error against
                the FP64 result, measured outside the timed region;
  per_stencil   every other workload of the study (25-point constant 512^3,
                25-point variable 384^3, 7-point variable 256x512x1024, the
                second-order 25-point stencil on 512^3, the 27-point box
                stencil on 512^3), blocked
                and naive, FP64 and FP32, timed the same way outside the timed
                region, with the FP32 error against the FP64 blocked result
                (which equals the FP64 oracle bit for bit, as the GPU parity
                tests check).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
WORKLOAD = "7pt-const-512"
STENCIL_NAMES = {"7c": "7-point constant (c0=0.4, c1=0.1)", "25c": "25-point constant (c0..c4 drawn, normalised)",
                 "7v": "7-point variable (7 coefficient arrays)", "25v": "25-point variable (13 coefficient arrays)",
                 "25l": "25-point second order in time (c0..c4, C array)",
                 "27b": "27-point box (c0..c3 by distance class)"}
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "mwd_7pt_const_512_f64_traffic.txt")
KERNEL_SOURCES = ("paper_1510_04995_amd/csrc/mwd.hpp", "paper_1510_04995_amd/csrc/lanes.hpp",
                  "paper_1510_04995_amd/csrc/stencils.hpp",
                  "paper_1510_04995_amd/csrc/kernels_7c_f64.hip", "paper_1510_04995_amd/csrc/instantiate.hpp")


def _code_only(text):
    """The source without // comments and blank lines, each line stripped, so
    that edits of comments do not change the hash (none of these sources puts
    // inside a string)."""
    out = []
    for line in text.splitlines():
        code = line.split("//", 1)[0].strip()
        if code:
            out.append(code)
    return "\n".join(out)


def kernel_source_hash():
    """Hash of the code of the diamond-row kernel's sources (comments excluded):
    a stored profile counts for this kernel only if its hash matches."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel)) as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def launch_lups(nx, ny, nz, T, H):
    """Lattice updates of each diamond-row launch: row r covers time steps
    [t_c - H, t_c + H) with t_c = r*H, each cell once per step it covers,
    clipped to [0, T); half of each row's diamonds cover each step."""
    n_rows = (T - 1) // H + 2
    out = []
    for r in range(n_rows):
        t_c = r * H
        steps = 0
        for s in range(t_c - H, t_c + H):
            if 0 <= s < T:
                steps += 1
        out.append(nx * ny * nz * steps / 2.0)
    return out


def x_halo_factor(q, R):
    """Cells an x chunk reads per cell it owns: the owned tile plus the
    redundant halo of R*(L-1) cells per side that the chunk recomputes."""
    L = q["diamond_width"] // R
    return (q["tile_x"] + 2 * R * (L - 1)) / q["tile_x"]


def host_info():
    """CPU model, sockets, logical CPUs, memory and C compiler of this host."""
    import platform
    import subprocess
    model, sockets = platform.processor() or "unknown", set()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                if k.strip() == "model name":
                    model = v.strip()
                elif k.strip() == "physical id":
                    sockets.add(v.strip())
    except OSError:
        pass
    mem_gb = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal:"):
                    mem_gb = round(int(line.split()[1]) / 2 ** 20, 1)
    except OSError:
        pass
    try:
        cc = subprocess.run(["gcc", "--version"], capture_output=True, text=True).stdout.splitlines()[0]
    except (OSError, IndexError):
        cc = "unknown"
    return {"cpu_model": model, "sockets": max(1, len(sockets)), "logical_cpus": os.cpu_count(),
            "mem_gib": mem_gb, "compiler": cc + " -O2 -ffp-contract=off -fopenmp"}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def time_runs(sw, g0, T, coefs, reps, torch):
    """Median seconds of `reps` runs of a plan from a fresh copy of g0 (HIP
    events on the current stream; the copies are outside the events)."""
    stream = torch.cuda.current_stream()
    b0, b1 = g0.clone(), g0.clone()
    sw.run(b0, b1, T, coefs)   # warm-up
    times = []
    for _ in range(reps):
        b0.copy_(g0)
        b1.copy_(g0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        out = sw.run(b0, b1, T, coefs)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    return sorted(times)[len(times) // 2], out


def per_stencil(torch, dev, reps=3):
    """The other workloads, blocked and naive, FP64 and FP32 (default plans)."""
    import numpy as np
    import paper_1510_04995_amd as P
    from workloads import WORKLOADS, field_and_coefs
    res = {}
    for name in ("25pt-const-512", "25pt-var-384", "7pt-var-256x512x1024", "25pt-leapfrog-512", "27pt-box-512"):
        w = WORKLOADS[name]
        h = w.radius
        algos = ("mwd", "naive")
        log("inputs " + name)
        u0, c, arr = field_and_coefs(w.stencil, w.nx, w.ny, w.nz, seed=0)
        consts = None if c is None else [float(x) for x in c]
        entry = {"stencil": w.stencil, "grid": [w.nx, w.ny, w.nz], "T": w.T}
        ref64 = None
        for dtype in ("f64", "f32"):
            npdt = np.float64 if dtype == "f64" else np.float32
            g0 = torch.from_numpy(u0.astype(npdt)).to(dev)
            coefs = [] if arr is None else [torch.from_numpy(a.astype(npdt)).to(dev) for a in arr]
            for algo in algos:
                log("time %s %s %s" % (name, dtype, algo))
                sw = P.Sweep(w.stencil, dtype, w.nx, w.ny, w.nz, consts, algo)
                info = sw.info()
                sec, out = time_runs(sw, g0, w.T, coefs, reps, torch)
                key = "%s_%s" % (algo, dtype)
                entry[key + "_glups"] = round(w.lups / sec / 1e9, 2)
                entry[key + "_bytes_per_lup_alg"] = round(info["model_bytes_per_lup"], 3)
                if algo == "mwd":
                    p = info["params"]
                    entry[key + "_plan"] = [p["diamond_width"], p["cells_per_lane"], p["threads_x"] // 64,
                                            p["tile_x"]]
                    if dtype == "f64":
                        ref64 = out.clone()
                    else:
                        rel, mx, _ = P.error_norms(out, ref64, h, w.nx, w.ny, w.nz)
                        entry["f32_rel_l2_vs_f64"] = float("%.3e" % rel)
                        entry["f32_max_abs_vs_f64"] = float("%.3e" % mx)
                else:
                    ref = ref64 if dtype == "f64" else None
                    if ref is not None:
                        entry["mwd_vs_naive_f64_bitwise_diff"] = P.error_norms(out, ref, h, w.nx, w.ny, w.nz)[2]
                    elif dtype == "f64":
                        ref64 = out.clone()
                    elif "mwd" not in algos:
                        rel, mx, _ = P.error_norms(out, ref64, h, w.nx, w.ny, w.nz)
                        entry["f32_rel_l2_vs_f64"] = float("%.3e" % rel)
                        entry["f32_max_abs_vs_f64"] = float("%.3e" % mx)
                sw.close()
                del out
            del g0, coefs
            torch.cuda.empty_cache()
        if "mwd" in algos:
            entry["mwd_vs_naive_f64"] = round(entry["mwd_f64_glups"] / entry["naive_f64_glups"], 3)
        del ref64
        torch.cuda.empty_cache()
        res[name] = entry
    return res


def oracle_rates(O, seconds=4.0):
    """The oracle on the other workloads: a few steps each on all threads."""
    from workloads import WORKLOADS, field_and_coefs
    out = {}
    for name in ("25pt-const-512", "25pt-var-384", "7pt-var-256x512x1024", "25pt-leapfrog-512", "27pt-box-512"):
        w = WORKLOADS[name]
        log("oracle " + name)
        u0, c, arr = field_and_coefs(w.stencil, w.nx, w.ny, w.nz, seed=0)
        a0, a1 = u0.copy(), u0.copy()
        t = time.perf_counter()
        O.sweep(w.stencil, a0, a1, 1, c, arr)
        one = time.perf_counter() - t
        steps = int(max(1, min(w.T, seconds / max(one, 1e-3))))
        a0, a1 = u0.copy(), u0.copy()
        t = time.perf_counter()
        O.sweep(w.stencil, a0, a1, steps, c, arr)
        dt = time.perf_counter() - t
        out[name] = {"glups": round(w.nx * w.ny * w.nz * steps / dt / 1e9, 4),
                     "sample": "%d of %d steps, %.1f s" % (steps, w.T, dt)}
        del a0, a1, u0, arr
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--params", default=None, help="JSON dict of girih_params fields for the blocked plan")
    ap.add_argument("--no-compare", action="store_true", help="skip the naive / FP32 comparison runs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-suite", action="store_true", help="skip the other workloads (per_stencil)")
    ap.add_argument("--workload", default=WORKLOAD,
                    help="workload of the timed runs (default: the headline 7-point constant 512^3; any other "
                         "workload serves profiling runs of its blocked kernel)")
    ap.add_argument("--dtype", default="f64", choices=("f64", "f32"),
                    help="element type of the timed runs (FP64 unless profiling the FP32 kernels)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also copy a buffer of this many MiB (a known-size reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the sweep is a single-device kernel here and no multi-GPU "
              "path is built (requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1510_04995_amd as P
    from workloads import WORKLOADS, field_and_coefs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    w = WORKLOADS[args.workload]
    if w.stencil not in ("7c", "25c", "7v", "25v", "25l", "27b"):
        print("unknown stencil of workload %s" % w.name, file=sys.stderr)
        sys.exit(2)
    if args.dtype != "f64" and (not args.no_compare or not args.no_cpu):
        print("--dtype f32 is for profiling runs (with --no-compare --no-cpu)", file=sys.stderr)
        sys.exit(2)
    h = w.radius
    u0, c, arr = field_and_coefs(w.stencil, w.nx, w.ny, w.nz, seed=0, const_coefs=w.const_coefs)
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    g0 = torch.from_numpy(u0).to(dev).to(tdt)
    coefs = [torch.from_numpy(a).to(dev).to(tdt) for a in (arr or [])]
    cl = None if c is None else list(c)
    params = json.loads(args.params) if args.params else None

    sw = P.Sweep(w.stencil, args.dtype, w.nx, w.ny, w.nz, cl, "mwd", params)
    info = sw.info()
    b0, b1 = g0.clone(), g0.clone()
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        sw.run(b0, b1, w.T, coefs)
    torch.cuda.synchronize()

    sw.set_timing(True)
    n_launch = 0
    kern_ms = 0.0
    times = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        sw.run(b0, b1, w.T, coefs)
        ev1.record(stream)
        ev1.synchronize()
        times.append(ev0.elapsed_time(ev1) * 1e-3)
        n, ms = sw.timing()   # events of this run, already complete
        n_launch += n
        kern_ms += ms
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sw.set_timing(False)

    lups = w.nx * w.ny * w.nz * w.T
    ms_per_step = wall / args.steps * 1e3
    value = lups * args.steps / wall / 1e9

    # roofline of the diamond-row kernel
    q = info["params"]
    H = q["diamond_width"] // (2 * h)
    # one launch per diamond row, or one dependency-driven launch per run
    sweep_launch = (q.get("variant", 0) & 1) == 1
    per_launch = [float(w.lups)] if sweep_launch else launch_lups(w.nx, w.ny, w.nz, w.T, H)
    bpl = info["model_bytes_per_lup"]   # the paper's B_C for this plan
    alg_bytes_per_launch = bpl * sum(per_launch) / len(per_launch)
    avg_launch_s = kern_ms / max(n_launch, 1) * 1e-3
    achieved = alg_bytes_per_launch / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
    traffic = None
    src_hash = kernel_source_hash()
    if os.path.exists(PROFILE_TRAFFIC):
        with open(PROFILE_TRAFFIC) as f:
            prof = json.load(f)
        if prof.get("kernel_source_hash") == src_hash and prof.get("params") == {
                k: q[k] for k in ("diamond_width", "tile_x", "threads_x", "cells_per_lane")}:
            traffic = prof.get("hbm_bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "mwd_sweep_kernel" if sweep_launch else "mwd_row_kernel",
                "bytes_per_lup_alg": round(bpl, 3),
                "x_halo_read_factor": round(x_halo_factor(q, h), 4),
                "traffic_vs_alg": None if traffic is None else round(traffic / alg_bytes_per_launch, 3),
                "lups_per_launch": round(sum(per_launch) / len(per_launch)), "launches": n_launch,
                "avg_launch_ms": round(avg_launch_s * 1e3, 4)}

    compare = None
    if not args.no_compare:
        compare = {}
        nv = P.Sweep(w.stencil, "f64", w.nx, w.ny, w.nz, cl, "naive")
        n0, n1 = g0.clone(), g0.clone()
        nv.run(n0, n1, w.T, coefs)
        torch.cuda.synchronize()
        t = time.perf_counter()
        reps = 3
        for _ in range(reps):
            ref = nv.run(n0, n1, w.T, coefs)
        torch.cuda.synchronize()
        compare["naive_f64_glups"] = round(lups * reps / (time.perf_counter() - t) / 1e9, 2)
        # bit-exactness of the blocked run on the same input
        m0, m1 = g0.clone(), g0.clone()
        res64 = sw.run(m0, m1, w.T, coefs)
        r0, r1 = g0.clone(), g0.clone()
        ref = nv.run(r0, r1, w.T, coefs)
        rel, mx, nd = P.error_norms(res64, ref, h, w.nx, w.ny, w.nz)
        compare["blocked_vs_naive_f64_bitwise_diff"] = nd
        nv.close()
        del n0, n1, r0, r1
        s32 = P.Sweep(w.stencil, "f32", w.nx, w.ny, w.nz, cl, "mwd")
        g32 = g0.to(torch.float32)
        c32 = [a.to(torch.float32) for a in coefs]
        f0, f1 = g32.clone(), g32.clone()
        s32.run(f0, f1, w.T, c32)
        best = None
        for _ in range(reps):
            # fresh input each time: the last run's result is the FP32 answer for u0
            f0.copy_(g32)
            f1.copy_(g32)
            torch.cuda.synchronize()
            t = time.perf_counter()
            res32 = s32.run(f0, f1, w.T, c32)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            best = dt if best is None else min(best, dt)
        compare["blocked_f32_glups"] = round(lups / best / 1e9, 2)
        rel32, mx32, _ = P.error_norms(res32, res64, h, w.nx, w.ny, w.nz)
        compare["f32_rel_l2_vs_f64"] = float("%.3e" % rel32)
        compare["f32_max_abs_vs_f64"] = float("%.3e" % mx32)
        compare["f32_params"] = s32.info()["params"]
        s32.close()
        del f0, f1, g32, m0, m1

    sw_rest = None
    if not args.no_suite:
        sw_rest = per_stencil(torch, dev)

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if not args.no_cpu:
        from oracle import sweep as O
        a0 = u0.copy()
        a1 = u0.copy()
        t = time.perf_counter()
        O.sweep(w.stencil, a0, a1, 2, c, arr)
        rate = w.nx * w.ny * w.nz * 2 / (time.perf_counter() - t)
        # about ten seconds of oracle time: the whole run when it is shorter
        # (repeated, continuing in time), else part of it
        t_s = int(max(2, 10.0 * rate / (w.nx * w.ny * w.nz)))
        a0 = u0.copy()
        a1 = u0.copy()
        t = time.perf_counter()
        O.sweep(w.stencil, a0, a1, t_s, c, arr)
        dt = time.perf_counter() - t
        what = ("%d of the %d steps" % (t_s, w.T) if t_s < w.T else
                "%d steps (the %d-step run %.1f times over)" % (t_s, w.T, t_s / w.T))
        cpu = {"value": round(w.nx * w.ny * w.nz * t_s / dt / 1e9, 4), "unit": "GLUP/s", "cores": O.num_threads(),
               "kind": "oracle",
               "sample": "%dx%dx%d %s FP64, %s, plain C sweep (OpenMP over z), %.1f s"
                         % (w.nx, w.ny, w.nz, STENCIL_NAMES[w.stencil], what, dt)}
        # the same sweep on one thread, about five seconds of it
        n_all = O.num_threads()
        O.set_num_threads(1)
        try:
            t1 = max(1, int(5.0 * cpu["value"] * 1e9 / n_all / (w.nx * w.ny * w.nz)))
            a0 = u0.copy()
            a1 = u0.copy()
            t = time.perf_counter()
            O.sweep(w.stencil, a0, a1, t1, c, arr)
            dt1 = time.perf_counter() - t
        finally:
            O.set_num_threads(n_all)
        cpu["value_one_thread"] = round(w.nx * w.ny * w.nz * t1 / dt1 / 1e9, 4)
        cpu["sample_one_thread"] = "%d steps, %.1f s" % (t1, dt1)
        cpu["host"] = host_info()
        if not args.no_suite:
            cpu["other_workloads"] = oracle_rates(O)

    out = {
        "metric": "GLUP/s per stencil at 1 GPU + % HBM roofline; blocked vs naive, FP32 vs FP64",
        "value": round(value, 2),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": w.name, "stencil": STENCIL_NAMES[w.stencil], "stencil_id": w.stencil,
                   "grid": [w.nx, w.ny, w.nz], "halo": h, "T": w.T, "algo": "mwd", "params": q,
                   "lds_bytes": info["lds_bytes"], "median_run_ms": round(sorted(times)[len(times) // 2] * 1e3, 3),
                   "kernel_source_hash": src_hash},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "compare": compare,
        "per_stencil": sw_rest,
    }
    print(json.dumps(out), flush=True)
    sw.close()


if __name__ == "__main__":
    main()
