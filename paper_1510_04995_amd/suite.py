"""Throughput of every workload of the study, naive and blocked, FP64 and FP32.

  python -m paper_1510_04995_amd.suite run [--reps 3]
      one JSON line per (workload, dtype, algorithm): GLUP/s (best of the
      timed runs, inputs resident on the device), the plan, its modelled bytes
      per update, and the checks: the blocked FP64 result against the naive
      FP64 result (elements that differ in any bit), and every FP32 result's
      relative L2 and largest absolute error against the naive FP64 result
      (the GPU naive sweep equals the oracle bit for bit, which the parity
      tests check).

  python -m paper_1510_04995_amd.suite summary <run.log> <out.md> <command...>
      a markdown table of those lines, with each rate next to the naive
      sweep's HBM roofline (domain-sized streams x element bytes per update at
      8 TB/s: the field read and written, the coefficient arrays, and for the
      second-order-in-time stencil the previous level read as well).

One more case is
one GPU's share of the 512^3 7-point problem split in y across two GPUs
(512 x 256 x 512), the shape a y-slab decomposition gives each device.
"""
import json
import sys
import time

HBM_PEAK_BYTES = 8.0e12
STREAMS = {"7c": 2, "7v": 9, "25c": 2, "25v": 15, "25l": 4, "27b": 2}


def _grid(a, torch, dev):
    return torch.from_numpy(a).to(dev)


def run(reps):
    import numpy as np
    import torch
    from . import Sweep, error_norms
    from workloads import WORKLOADS, Workload, field_and_coefs
    dev = torch.device("cuda:0")
    # a device-to-device copy of 2 GiB: the HBM rate a streaming kernel reaches
    src = torch.ones(1 << 28, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = None
    for _ in range(5):
        t = time.perf_counter()
        dst.copy_(src)
        torch.cuda.synchronize()
        dtm = time.perf_counter() - t
        best = dtm if best is None else min(best, dtm)
    print(json.dumps({"workload": "device-copy", "bytes": 2 * src.numel() * 8, "seconds": best,
                      "gb_per_s": 2 * src.numel() * 8 / best * 1e-9}), flush=True)
    del src, dst
    cases = dict(WORKLOADS)
    base = WORKLOADS["7pt-const-512"]
    cases["7pt-const-512-yhalf"] = Workload("7pt-const-512-yhalf", "7c", base.nx, base.ny // 2, base.nz, base.T,
                                            base.const_coefs, ("f64",), note="one GPU's y-slab of 7pt-const-512")
    for name, w in cases.items():
        h = w.radius
        u0, c, arr = field_and_coefs(w.stencil, w.nx, w.ny, w.nz, seed=0, const_coefs=w.const_coefs)
        consts = None if c is None else [float(x) for x in c]
        ref = None
        algos = ("naive", "mwd")
        for dt in w.dtypes:
            npdt = np.float64 if dt == "f64" else np.float32
            g0 = _grid(u0.astype(npdt), torch, dev)
            coefs = [] if arr is None else [_grid(a.astype(npdt), torch, dev) for a in arr]
            for algo in algos:
                sw = Sweep(w.stencil, dt, w.nx, w.ny, w.nz, consts, algo)
                info = sw.info()
                b0, b1 = g0.clone(), g0.clone()
                sw.run(b0, b1, w.T, coefs)          # warm-up
                torch.cuda.synchronize()
                best = None
                for _ in range(reps):
                    b0.copy_(g0)
                    b1.copy_(g0)
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    out = sw.run(b0, b1, w.T, coefs)
                    torch.cuda.synchronize()
                    dtm = time.perf_counter() - t
                    best = dtm if best is None else min(best, dtm)
                rec = {"workload": name, "stencil": w.stencil, "grid": [w.nx, w.ny, w.nz], "T": w.T,
                       "dtype": dt, "algo": algo, "glups": w.lups / best * 1e-9, "seconds": best,
                       "model_bytes_per_lup": info["model_bytes_per_lup"],
                       "params": {k: info["params"][k] for k in ("diamond_width", "tile_x", "threads_x",
                                                                 "cells_per_lane")}}
                if dt == "f64" and algo == "naive":
                    ref = out.clone()
                elif dt == "f64":
                    _, _, nd = error_norms(out, ref, h, w.nx, w.ny, w.nz)
                    rec["bitwise_diff_vs_naive_f64"] = nd
                if dt == "f32" and ref is not None:
                    rel, mx, _ = error_norms(out, ref, h, w.nx, w.ny, w.nz)
                    rec["rel_l2_vs_f64"] = rel
                    rec["max_abs_vs_f64"] = mx
                print(json.dumps(rec), flush=True)
                sw.close()
                del b0, b1, out
            del g0, coefs
            torch.cuda.empty_cache()
        ref = None
        torch.cuda.empty_cache()


def summary(run_log, out_path, command):
    recs = [json.loads(l) for l in open(run_log) if l.startswith("{")]
    copy = [r for r in recs if r["workload"] == "device-copy"]
    recs = [r for r in recs if r["workload"] != "device-copy"]
    lines = ["# Throughput of the study's workloads", "",
             "Command: `%s`" % command, "",
             "GLUP/s = nx*ny*nz*T / best of the timed runs (inputs resident in HBM).  Naive roofline: "
             "domain-sized streams (field read + written, coefficient arrays, previous level for 25l) x element "
             "bytes per update at 8 TB/s.  Checks against the naive FP64 result: "
             "blocked FP64 elements differing in any bit; FP32 relative L2 / max abs error.", "",
             "| workload | dtype | sweep | GLUP/s | naive roofline | model B/update | plan (Dw, x tile, threads_x, "
             "cells/lane) | check |", "|---|---|---|---|---|---|---|---|"]
    if copy:
        lines.insert(5, "A 2 GiB device-to-device copy runs at %.0f GB/s (read + write)." % copy[0]["gb_per_s"])
        lines.insert(6, "")
    for r in recs:
        s = 8 if r["dtype"] == "f64" else 4
        roof = HBM_PEAK_BYTES / (STREAMS[r["stencil"]] * s) * 1e-9
        q = r["params"]
        plan = "-" if r["algo"] == "naive" else "%d, %d, %d, %d" % (q["diamond_width"], q["tile_x"], q["threads_x"],
                                                                    q["cells_per_lane"])
        if "bitwise_diff_vs_naive_f64" in r:
            chk = "%d differ" % r["bitwise_diff_vs_naive_f64"]
        elif "rel_l2_vs_f64" in r:
            chk = "%.2e / %.2e" % (r["rel_l2_vs_f64"], r["max_abs_vs_f64"])
        else:
            chk = "reference"
        lines.append("| %s | %s | %s | %.1f | %.0f | %.2f | %s | %s |" % (
            r["workload"], r["dtype"], r["algo"], r["glups"], roof, r["model_bytes_per_lup"], plan, chk))
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "run":
        reps = 3
        if "--reps" in sys.argv:
            reps = int(sys.argv[sys.argv.index("--reps") + 1])
        run(reps)
    elif len(sys.argv) > 1 and sys.argv[1] == "summary":
        summary(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
    else:
        raise SystemExit(__doc__)
