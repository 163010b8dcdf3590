"""Summaries of rocprofv3 output for the benchmark's roofline figures.

  python -m paper_1510_04995_amd.profsum stats <kernel_stats.csv> <bench.json> <out.md> <command...>
      kernel-trace statistics (calls, average duration) as a short table.

  python -m paper_1510_04995_amd.profsum traffic <fetch.csv> <write.csv> <bench.json> <copy_mib> <out.json> <command...>
      HBM bytes per launch of the diamond-row kernel from two counter runs
      (FETCH_SIZE, WRITE_SIZE: KiB per dispatch), each scaled by what the same
      counter reads for a device-to-device copy of copy_mib MiB in the same run.

<bench.json> is the JSON line bench.py printed in the profiled run (its plan
parameters and kernel source hash are recorded with the numbers).
"""
import csv
import json
import sys

ROW_KERNEL = "mwd_row_kernel"
COPY_KERNEL = "copyBuffer"


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
    key = "%s, %d, %d, %d," % ("double" if b["dtype"] == "f64" else "float", q["diamond_width"],
                               q["cells_per_lane"], q["threads_x"] // 64)
    mine = [r for r in rows if ROW_KERNEL in r["Name"] and key in r["Name"]]
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
        rows = [v for (k, _), v in d.items() if ROW_KERNEL in k]
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
        res["bytes_per_lup_model"] = rl["bytes_per_lup_model"]
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4], " ".join(sys.argv[5:]))
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6], " ".join(sys.argv[7:]))
    else:
        raise SystemExit(__doc__)
