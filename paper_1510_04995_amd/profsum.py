"""Summaries of rocprofv3 output for the benchmark's roofline figures.

  python -m paper_1510_04995_amd.profsum stats <kernel_stats.csv> <bench.json> <out.md> <command...>
      kernel-trace statistics (calls, average duration) as a short table.

  python -m paper_1510_04995_amd.profsum traffic <fetch.csv> <write.csv> <bench.json> <copy_mib> <out.json> <command...>
      HBM bytes per launch of the diamond-row kernel from two counter runs
      (FETCH_SIZE, WRITE_SIZE: KiB per dispatch), each scaled by what the same
      counter reads for a device-to-device copy of copy_mib MiB in the same run.

  python -m paper_1510_04995_amd.profsum core <pass_a.csv> <pass_b.csv> <bench.json> <out.md> <command...>
      in-core utilisation of the diamond-row kernel from two SQ counter runs:
      VALU busy, FP64 rate, LDS busy and bytes, against the CU count, clock
      and peaks of the chip.

<bench.json> is the JSON line bench.py printed in the profiled run (its plan
parameters and kernel source hash are recorded with the numbers).
"""
import csv
import json
import sys

ROW_KERNEL = "mwd_row_kernel"
SWEEP_KERNEL = "mwd_sweep_kernel"


def _kernel_of(b):
    """Name stem of the bench line's dominant kernel (row launches or the
    dependency-driven whole-sweep launch)."""
    return b.get("roofline", {}).get("kernel", ROW_KERNEL)
COPY_KERNEL = "copyBuffer"
# MI355X: 256 CUs of 4 SIMDs in 8 XCDs; FP64 vector peak 78.6 TFLOP/s; LDS
# 128 bytes per clock per CU
N_CU, N_SIMD, N_XCD = 256, 1024, 8
FP64_PEAK_TFLOPS = 78.6
LDS_BYTES_PER_CLK = 128


STENCIL_CLASS = {"7c": "Stencil7C", "7v": "Stencil7V", "25c": "Stencil25C", "25v": "Stencil25V", "25l": "Stencil25L",
                 "27b": "Stencil27B"}


def _plan_key(b):
    """The part of the diamond-row kernel's name that identifies the bench
    line's plan (stencil, element type, diamond width, cells per lane, waves
    along x), shared by its full and clipped-row instances."""
    q = b["config"]["params"]
    st = STENCIL_CLASS[b["config"].get("stencil_id", "7c")]
    return "%s, %s, %d, %d, %d," % (st, "double" if b["dtype"] == "f64" else "float", q["diamond_width"],
                                    q["cells_per_lane"], q["threads_x"] // 64)


def _bench_line(path):
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("{") and '"metric"' in line:
                return json.loads(line)
    raise ValueError("no bench.py JSON line in %s" % path)


def stats(csv_path, bench_path, out_path, command):
    b = _bench_line(bench_path)
    rows = list(csv.DictReader(open(csv_path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# Kernel time, %s" % b["config"]["workload"], "",
             "Command: `%s`" % command, "",
             "Plan: %s" % json.dumps({k: b["config"]["params"][k] for k in
                                      ("diamond_width", "tile_x", "threads_x", "cells_per_lane")}),
             "Kernel source hash: %s" % b["config"]["kernel_source_hash"], "",
             "| kernel | calls | total ms | average us | share % |", "|---|---|---|---|---|"]
    for r in rows[:8]:
        name = r["Name"]
        short = name.split("(")[0][:90]
        lines.append("| %s | %s | %.3f | %.2f | %.1f |" % (short, r["Calls"], float(r["TotalDurationNs"]) * 1e-6,
                                                          float(r["AverageNs"]) * 1e-3, float(r["Percentage"])))
    # the plan's diamond-row kernels (full and clipped-row slot counts) together:
    # bench.py's per-launch average covers all of them
    q = b["config"]["params"]
    key = _plan_key(b)
    mine = [r for r in rows if _kernel_of(b) in r["Name"] and key in r["Name"]]
    calls = sum(int(r["Calls"]) for r in mine)
    tot_ns = sum(float(r["TotalDurationNs"]) for r in mine)
    rl = b["roofline"]
    if calls:
        lines += ["", "Plan's diamond-row kernels together (%d variants): %d calls, average %.2f us" %
                  (len(mine), calls, tot_ns / calls * 1e-3)]
    lines += ["", "bench.py (same run, HIP events on the launch stream): %d launches, average %.4f ms; "
              "value %.2f GLUP/s" % (rl["launches"], rl["avg_launch_ms"], b["value"])]
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


def _per_dispatch(csv_path, counter):
    """{(kernel name, dispatch id): counter value summed over its rows}."""
    out = {}
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] != counter:
            continue
        key = (r["Kernel_Name"], int(r["Dispatch_Id"]))
        out[key] = out.get(key, 0.0) + float(r["Counter_Value"])
    return out


def traffic(fetch_csv, write_csv, bench_path, copy_mib, out_path, command):
    b = _bench_line(bench_path)
    copy_kib = float(copy_mib) * 1024.0
    res = {"command": command, "kernel_source_hash": b["config"]["kernel_source_hash"],
           "params": {k: b["config"]["params"][k] for k in ("diamond_width", "tile_x", "threads_x", "cells_per_lane")},
           "workload": b["config"]["workload"], "copy_probe_mib": float(copy_mib)}
    total = 0.0
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        d = _per_dispatch(path, counter)
        copies = sorted((i, v) for (k, i), v in d.items() if COPY_KERNEL in k)
        # the probe is the last copy of the run (bench.py issues it after the sweeps)
        probe = copies[-1][1] if copies else None
        rows = [v for (k, _), v in d.items() if _kernel_of(b) in k]
        scale = copy_kib / probe if probe else None
        mean_kib = sum(rows) / len(rows) if rows else None
        res[counter] = {"row_kernel_dispatches": len(rows), "row_kernel_mean_kib": mean_kib,
                        "copy_probe_kib_counted": probe, "scale": scale,
                        "row_kernel_bytes_per_launch": mean_kib * 1024.0 * scale if (mean_kib and scale) else None}
        if res[counter]["row_kernel_bytes_per_launch"]:
            total += res[counter]["row_kernel_bytes_per_launch"]
    res["hbm_bytes_per_launch"] = total or None
    rl = b["roofline"]
    if total:
        res["bytes_per_lup_measured"] = total / rl["lups_per_launch"]
        res["bytes_per_lup_alg"] = rl["bytes_per_lup_alg"]
        res["x_halo_read_factor"] = rl.get("x_halo_read_factor")
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
        f.write("\n")


def _row_kernel_means(path, key, kernel=ROW_KERNEL):
    """{counter: mean over the plan's dispatches of `kernel` of the per-dispatch sum}."""
    per = {}
    for r in csv.DictReader(open(path)):
        if kernel not in r["Kernel_Name"] or key not in r["Kernel_Name"]:
            continue
        k = (r["Counter_Name"], int(r["Dispatch_Id"]))
        per[k] = per.get(k, 0.0) + float(r["Counter_Value"])
        per[("_ns", int(r["Dispatch_Id"]))] = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
    out = {}
    for (c, _), v in per.items():
        out.setdefault(c, []).append(v)
    return {c: sum(v) / len(v) for c, v in out.items()}


def core(path_a, path_b, bench_path, out_path, command):
    b = _bench_line(bench_path)
    q = b["config"]["params"]
    key = _plan_key(b)
    m = _row_kernel_means(path_a, key, _kernel_of(b))
    m.update({k: v for k, v in _row_kernel_means(path_b, key, _kernel_of(b)).items() if k not in m})
    cyc = m["GRBM_GUI_ACTIVE"] / N_XCD              # kernel cycles (the counter sums the XCDs)
    ns = m["_ns"]
    clock_ghz = cyc / ns
    simd_cycles = N_SIMD * cyc
    valu_busy = 4.0 * m["SQ_ACTIVE_INST_VALU"] / simd_cycles   # a wave64 VALU instruction: 4 cycles of a SIMD
    fp64_flops = 64.0 * (m["SQ_INSTS_VALU_ADD_F64"] + m["SQ_INSTS_VALU_MUL_F64"])
    fp64_tflops = fp64_flops / ns * 1e-3
    lds_busy = m["SQ_LDS_IDX_ACTIVE"] / (N_CU * cyc)
    lds_bytes = 64.0 * (m["SQ_INSTS_LDS_LOAD_BANDWIDTH"] + m["SQ_INSTS_LDS_STORE_BANDWIDTH"])
    lds_bw = lds_bytes / (N_CU * cyc)
    waves = m["SQ_WAVES"]
    rl = b["roofline"]
    rows = [("kernel duration (counter run, mean over the plan's row launches)", "%.3f ms" % (ns * 1e-6)),
            ("shader clock (GRBM_GUI_ACTIVE / duration)", "%.2f GHz" % clock_ghz),
            ("waves per launch", "%.0f" % waves),
            ("VALU busy, all 1024 SIMDs (4 x SQ_ACTIVE_INST_VALU / SIMD cycles)", "%.1f %%" % (100 * valu_busy)),
            ("VALU instructions per wave", "%.0f" % (m["SQ_INSTS_VALU"] / waves)),
            ("FP64 add+mul instructions / VALU instructions", "%.1f %%" % (
                100 * (m["SQ_INSTS_VALU_ADD_F64"] + m["SQ_INSTS_VALU_MUL_F64"]) / m["SQ_INSTS_VALU"])),
            ("FP64 rate (64 x add+mul instructions / duration)", "%.2f TFLOP/s = %.1f %% of %.1f" % (
                fp64_tflops, 100 * fp64_tflops / FP64_PEAK_TFLOPS, FP64_PEAK_TFLOPS)),
            ("LDS busy, all 256 CUs (SQ_LDS_IDX_ACTIVE / CU cycles)", "%.1f %%" % (100 * lds_busy)),
            ("LDS bytes per CU per clock (64 B x LDS load+store bandwidth units)", "%.1f of %d" % (
                lds_bw, LDS_BYTES_PER_CLK)),
            ("LDS bank conflicts (SQ_LDS_BANK_CONFLICT)", "%.0f" % m.get("SQ_LDS_BANK_CONFLICT", 0.0)),
            ("SALU instructions per wave", "%.0f" % (m["SQ_INSTS_SALU"] / waves)),
            ("LDS instructions per wave", "%.0f" % (m["SQ_INSTS_LDS"] / waves))]
    lines = ["# In-core utilisation, diamond-row kernel, %s" % b["config"]["workload"], "",
             "Command: `%s`" % command, "",
             "Plan: %s" % json.dumps({k: q[k] for k in ("diamond_width", "tile_x", "threads_x", "cells_per_lane")}),
             "Kernel source hash: %s" % b["config"]["kernel_source_hash"], "",
             "Means over the plan's diamond-row launches (both slot-count instances) of two SQ counter runs; "
             "chip totals: %d CUs, %d SIMDs, %d XCDs." % (N_CU, N_SIMD, N_XCD), "",
             "| quantity | value |", "|---|---|"]
    lines += ["| %s | %s |" % r for r in rows]
    lines += ["", "bench.py (same run): %.2f GLUP/s, %.1f %% of the HBM roofline at %.3f B/LUP (the paper's "
              "B_C of the plan)" % (b["value"], 100 * rl["frac"], rl["bytes_per_lup_alg"])]
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4], " ".join(sys.argv[5:]))
    elif sys.argv[1] == "core":
        core(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], " ".join(sys.argv[6:]))
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6], " ".join(sys.argv[7:]))
    else:
        raise SystemExit(__doc__)
