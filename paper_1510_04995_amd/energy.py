"""GPU energy per lattice update, blocked against naive (the paper's energy
versus code-balance discussion, on the GPU).

  python -m paper_1510_04995_amd.energy run [--seconds 6]
      for each case, repeats the sweep for about --seconds while a thread
      samples the socket power with `amd-smi metric -p --json`; one JSON line
      per case: GLUP/s, mean power over the samples taken after the first
      second, energy per update, and the idle power measured before the runs.

  python -m paper_1510_04995_amd.energy summary <run.log> <out.md> <command...>
      a markdown table of those lines.

The socket power is what the device's firmware reports (a short running
average); energy per update = mean power / update rate.
"""
import json
import subprocess
import sys
import threading
import time

CASES = [
    ("7c", "f64", (512, 512, 512), 64, "naive"),
    ("7c", "f64", (512, 512, 512), 64, "mwd"),
    ("7c", "f32", (512, 512, 512), 64, "naive"),
    ("7c", "f32", (512, 512, 512), 64, "mwd"),
    ("25c", "f64", (512, 512, 512), 32, "naive"),
    ("25c", "f64", (512, 512, 512), 32, "mwd"),
    ("27b", "f64", (512, 512, 512), 32, "naive"),
    ("27b", "f64", (512, 512, 512), 32, "mwd"),
    ("27b", "f32", (512, 512, 512), 32, "naive"),
    ("27b", "f32", (512, 512, 512), 32, "mwd"),
]
# the box stencil's weights are the workload recipe's (drawn and normalised)
CONSTS = {"7c": [0.4, 0.1], "25c": [0.2, 0.05, 0.04, 0.03, 0.0133], "27b": None}


def socket_power_w():
    """Socket power of GPU 0 in watts, or None if amd-smi does not report it."""
    try:
        out = subprocess.run(["amd-smi", "metric", "-p", "--json"], capture_output=True, text=True, timeout=20)
        d = json.loads(out.stdout)
        gpus = d["gpu_data"] if isinstance(d, dict) else d
        v = gpus[0]["power"]["socket_power"]["value"]
        return float(v)
    except (OSError, ValueError, KeyError, IndexError, TypeError, subprocess.SubprocessError):
        return None


class Sampler:
    def __init__(self, period=0.2):
        self.period = period
        self.samples = []
        self._stop = threading.Event()
        self._t = threading.Thread(target=self._loop, daemon=True)

    def _loop(self):
        while not self._stop.is_set():
            p = socket_power_w()
            if p is not None:
                self.samples.append((time.perf_counter(), p))
            self._stop.wait(self.period)

    def __enter__(self):
        self.t0 = time.perf_counter()
        self._t.start()
        return self

    def __exit__(self, *exc):
        self._stop.set()
        self._t.join()


def run(seconds):
    import torch
    from . import Sweep
    from workloads import field_and_coefs
    dev = torch.device("cuda:0")
    idle = [p for p in (socket_power_w() for _ in range(5)) if p is not None]
    print(json.dumps({"case": "idle", "power_w": sum(idle) / len(idle) if idle else None,
                      "samples": len(idle)}), flush=True)
    for st, dt, (nx, ny, nz), T, algo in CASES:
        u0, c, _ = field_and_coefs(st, nx, ny, nz, seed=0, const_coefs=CONSTS[st])
        g = torch.from_numpy(u0).to(dev)
        if dt == "f32":
            g = g.to(torch.float32)
        sw = Sweep(st, dt, nx, ny, nz, [float(x) for x in c], algo)
        b0, b1 = g.clone(), g.clone()
        sw.run(b0, b1, T)
        torch.cuda.synchronize()
        runs = 0
        with Sampler() as smp:
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < seconds:
                sw.run(b0, b1, T)
                torch.cuda.synchronize()
                runs += 1
            t1 = time.perf_counter()
        glups = nx * ny * nz * T * runs / (t1 - t0) * 1e-9
        steady = [p for (t, p) in smp.samples if t >= smp.t0 + 1.0 and t <= t1]
        pw = sum(steady) / len(steady) if steady else None
        q = sw.info()["params"]
        print(json.dumps({"case": "%s %s %s" % (st, dt, algo), "stencil": st, "dtype": dt, "algo": algo,
                          "grid": [nx, ny, nz], "T": T, "runs": runs, "glups": glups, "power_w": pw,
                          "samples": len(steady),
                          "nj_per_lup": pw / (glups * 1e9) * 1e9 if pw else None,
                          "params": {k: q[k] for k in ("diamond_width", "tile_x", "threads_x", "threads_y",
                                                       "cells_per_lane", "variant")}}), flush=True)
        sw.close()
        del b0, b1, g
        torch.cuda.empty_cache()


def summary(run_log, out_path, command):
    recs = [json.loads(l) for l in open(run_log) if l.startswith("{")]
    idle = [r for r in recs if r["case"] == "idle"]
    recs = [r for r in recs if r["case"] != "idle"]
    lines = ["# GPU energy per update, blocked against naive", "",
             "Command: `%s`" % command, "",
             "Socket power from `amd-smi metric -p` sampled every ~0.2 s while the sweep repeats; mean over "
             "the samples after the first second.  Idle power before the runs: %s W." % (
                 "%.0f" % idle[0]["power_w"] if idle and idle[0]["power_w"] else "n/a"), "",
             "| case | grid, T | GLUP/s | mean power W | samples | nJ per update |", "|---|---|---|---|---|---|"]
    for r in recs:
        lines.append("| %s | %s, %d | %.1f | %s | %d | %s |" % (
            r["case"], "x".join(str(v) for v in r["grid"]), r["T"], r["glups"],
            "%.0f" % r["power_w"] if r["power_w"] else "n/a", r["samples"],
            "%.3f" % r["nj_per_lup"] if r["nj_per_lup"] else "n/a"))
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "run":
        secs = 6.0
        if "--seconds" in sys.argv:
            secs = float(sys.argv[sys.argv.index("--seconds") + 1])
        run(secs)
    elif len(sys.argv) > 1 and sys.argv[1] == "summary":
        summary(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
    else:
        raise SystemExit(__doc__)
