"""Measured HBM bytes per lattice update against the traffic model, over
diamond widths and sweep kernels: the GPU counterpart of the paper's study of code balance
versus diamond width (Section "Memory traffic model" and the results that
compare measured and modelled bytes per update).

  python -m paper_1510_04995_amd.dw_sweep run [--copy-probe-mib 1024]
      runs every case once (one JSON line each: plan, model bytes per update,
      launches of the sweep kernel), then a device copy of known size;
      meant to run under rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE.

  python -m paper_1510_04995_amd.dw_sweep summary <fetch.csv> <write.csv> <run.log> <copy_mib> <out.md> <command...>
      bytes per update of every case from the two counter runs (KiB per
      dispatch, each scaled by what the counter reads for the copy), beside
      the model; a short markdown table.
"""
import csv
import json
import sys

CASES = [
    # (stencil, dtype, (nx, ny, nz), T, algo, params)
    ("7c", "f64", (512, 512, 512), 64, "naive", None),
    ("7c", "f64", (512, 512, 512), 64, "mwd", {"diamond_width": 4, "cells_per_lane": 2, "threads_x": 128}),
    ("7c", "f64", (512, 512, 512), 64, "mwd", {"diamond_width": 8, "cells_per_lane": 1, "threads_x": 128,
                                               "tile_x": 103}),
    ("7c", "f64", (512, 512, 512), 64, "mwd", {"diamond_width": 8, "cells_per_lane": 1, "threads_x": 192,
                                               "tile_x": 171}),
    ("7c", "f64", (512, 512, 512), 64, "mwd", {"diamond_width": 12, "cells_per_lane": 1, "threads_x": 128,
                                               "tile_x": 103}),
    ("7c", "f64", (512, 512, 512), 64, "mwd", {"diamond_width": 16, "cells_per_lane": 1, "threads_x": 64}),
    # FP32: the blocked sweep at the benchmark's plan against the naive sweep
    ("7c", "f32", (512, 512, 512), 64, "naive", None),
    ("7c", "f32", (512, 512, 512), 64, "mwd", {"diamond_width": 12, "cells_per_lane": 1, "threads_x": 128,
                                               "tile_x": 103}),
    ("25c", "f64", (512, 512, 512), 32, "naive", None),
    ("25c", "f64", (512, 512, 512), 32, "mwd", {"diamond_width": 8, "cells_per_lane": 1, "threads_x": 128}),
    ("25c", "f64", (512, 512, 512), 32, "mwd", {"diamond_width": 16, "cells_per_lane": 1, "threads_x": 64}),
    # the naive register columns (FP32 defaults of the star stencils) and the box stencil
    ("25c", "f32", (512, 512, 512), 32, "naive", None),
    ("27b", "f64", (512, 512, 512), 32, "naive", None),
    ("27b", "f32", (512, 512, 512), 32, "naive", None),
    ("27b", "f64", (512, 512, 512), 32, "mwd", None),
]
# the box stencil's weights are the workload recipe's (drawn and normalised)
CONSTS = {"7c": [0.4, 0.1], "25c": [0.2, 0.05, 0.04, 0.03, 0.0133], "27b": None}
SWEEP_KERNELS = ("mwd_row_kernel", "naive_step_kernel", "naive_tile_kernel", "naive_box_cols_kernel",
                 "naive_star_cols_kernel")
COPY_KERNEL = "copyBuffer"


def run(copy_mib):
    import torch
    from . import Sweep
    from workloads import field_and_coefs
    dev = torch.device("cuda:0")
    for st, dt, (nx, ny, nz), T, algo, prm in CASES:
        u0, c, _ = field_and_coefs(st, nx, ny, nz, seed=0, const_coefs=CONSTS[st])
        g = torch.from_numpy(u0).to(dev)
        if dt == "f32":
            g = g.to(torch.float32)
        sw = Sweep(st, dt, nx, ny, nz, [float(x) for x in c], algo, prm)
        info = sw.info()
        b0, b1 = g.clone(), g.clone()
        sw.run(b0, b1, T)
        torch.cuda.synchronize()
        q = info["params"]
        R = 4 if st.startswith("25") else 1
        launches = T if algo == "naive" else (T - 1) // (q["diamond_width"] // (2 * R)) + 2
        print(json.dumps({"stencil": st, "dtype": dt, "grid": [nx, ny, nz], "T": T, "algo": algo,
                          "params": {k: q[k] for k in ("diamond_width", "tile_x", "threads_x", "cells_per_lane")},
                          "model_bytes_per_lup": info["model_bytes_per_lup"], "launches": launches}), flush=True)
        sw.close()
        del b0, b1, g
    if copy_mib > 0:
        n = copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()


def _dispatches(path, counter):
    """[(dispatch id, kernel name, KiB)] in dispatch order."""
    d = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        key = int(r["Dispatch_Id"])
        name, v = d.get(key, (r["Kernel_Name"], 0.0))
        d[key] = (name, v + float(r["Counter_Value"]))
    return [(i, d[i][0], d[i][1]) for i in sorted(d)]


def summary(fetch_csv, write_csv, run_log, copy_mib, out_path, command):
    cases = [json.loads(l) for l in open(run_log) if l.startswith("{")]
    per = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        ds = _dispatches(path, counter)
        copies = [v for _, n, v in ds if COPY_KERNEL in n]
        scale = float(copy_mib) * 1024.0 / copies[-1]
        sweep = [v for _, n, v in ds if any(k in n for k in SWEEP_KERNELS)]
        need = sum(c["launches"] for c in cases)
        if len(sweep) != need:
            raise SystemExit("%s: %d sweep dispatches, expected %d" % (counter, len(sweep), need))
        i = 0
        for j, c in enumerate(cases):
            kib = sum(sweep[i:i + c["launches"]])
            i += c["launches"]
            per.setdefault(j, {})[counter] = kib * 1024.0 * scale
        per["scale_" + counter] = scale
    lines = ["# Measured HBM bytes per update against the model, over diamond widths and sweep kernels", "",
             "Command: `%s`" % command, "",
             "Counters `FETCH_SIZE` and `WRITE_SIZE` (KiB per dispatch) summed over every sweep launch of a case, "
             "each scaled by what it reads for a %s MiB device copy in the same run (factors %.3f and %.3f); "
             "updates = nx*ny*nz*T." % (copy_mib, per["scale_FETCH_SIZE"], per["scale_WRITE_SIZE"]), "",
             "| stencil | algo | Dw | x tile | threads_x | launches | measured B/update | model B/update |",
             "|---|---|---|---|---|---|---|---|"]
    for j, c in enumerate(cases):
        lups = c["grid"][0] * c["grid"][1] * c["grid"][2] * c["T"]
        meas = (per[j]["FETCH_SIZE"] + per[j]["WRITE_SIZE"]) / lups
        q = c["params"]
        lines.append("| %s %s | %s | %s | %s | %s | %d | %.2f | %.2f |" % (
            c["stencil"], c["dtype"], c["algo"], q["diamond_width"] or "-", q["tile_x"], q["threads_x"],
            c["launches"], meas, c["model_bytes_per_lup"]))
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "run":
        mib = 1024
        if "--copy-probe-mib" in sys.argv:
            mib = int(sys.argv[sys.argv.index("--copy-probe-mib") + 1])
        run(mib)
    elif len(sys.argv) > 1 and sys.argv[1] == "summary":
        summary(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6], " ".join(sys.argv[7:]))
    else:
        raise SystemExit(__doc__)
