"""Evaluation of the learned cost model against the paper's tuner.

  python -m paper_1510_04995_amd.tune_study [--out report.json] [--log train.jsonl]
  python -m paper_1510_04995_amd.tune_study summary <report.json> <out.md> <command...>
  python -m paper_1510_04995_amd.tune_study tgs <train.jsonl> <out.md> <command...>

1. The tuner measures every feasible blocked candidate (exhaustive search) of
   the training problems: 7-point constant 64^3 (T = 16) and 512^3 (T = 64),
   25-point constant 512^3 (T = 32) and 7-point variable 256^3 (T = 32),
   each in FP64 and FP32.  Every measured candidate is one training record
   (features, GLUP/s).
2. The cost model is trained on those records (HIP kernels, Adam).
3. On the problem the model has not seen -- the 7-point variable-coefficient
   stencil (seven coefficient arrays) on 256 x 512 x 1024, T = 64, in FP64
   and FP32, a grid and a step count none of the training problems has --
   and, as further unseen problems, the constant-coefficient stencils on
   the same grid, the study compares exhaustive search, the
   paper's hill-climbing tuner, the model's top-5 and the paper's "largest
   tile that fits" pick: best measured GLUP/s, number of candidates measured
   and tuning time.

Prints one progress line per problem and a JSON report at the end; the
`summary` form writes that report as a markdown table.  The `tgs` form
writes, from the training records, the GPU counterpart of the paper's
thread-group-size study: the best measured rate of each workgroup shape
(waves per tile = row pairs x waves along x, cells per lane), over diamond
widths, wavefront depths, x tiles and schedules.
"""
import argparse
import json
import sys
import time

import numpy as np

from . import Sweep
from . import costmodel as C

TRAIN = [("7c", (64, 64, 64), 16), ("7c", (512, 512, 512), 64), ("25c", (512, 512, 512), 32),
         ("7v", (256, 256, 256), 32)]
EVAL = [("7v", "f64"), ("7v", "f32"), ("7c", "f64"), ("7c", "f32"), ("25c", "f64")]
EVAL_GRID = (256, 512, 1024)
EVAL_T = 64
CONSTS = {"7c": [0.4, 0.1], "25c": [0.2, 0.05, 0.04, 0.03, 0.0133], "7v": None}


def say(*a):
    print(*a, flush=True)


def largest_tile_pick(sw, T):
    """The paper's capacity rule: the candidate with the largest diamond width,
    then the widest x tile, that the on-chip budget admits."""
    table = C.candidate_table(sw, T)
    best = max(table, key=lambda r: (r[0]["diamond_width"], r[0]["tile_x"] * 1.0, r[0]["threads_x"]))
    return best[0]


def timed_tune(sw, mode, T, budget, cands=None):
    if cands is not None:
        sw.set_candidates(cands)
    n0 = len(sw.tune_log())
    t0 = time.perf_counter()
    best, rate = sw.tune(mode, T, budget)
    return {"glups": rate, "measured": len(sw.tune_log()) - n0, "seconds": time.perf_counter() - t0,
            "params": {k: best[k] for k in ("diamond_width", "wavefront_depth", "tile_x", "threads_x", "cells_per_lane",
                                            "variant")}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--log", default=None, help="write the training records as JSON lines")
    ap.add_argument("--budget", type=float, default=60.0, help="seconds per exhaustive search")
    ap.add_argument("--constant-only", action="store_true",
                    help="train on the constant-coefficient problems only")
    args = ap.parse_args()

    train = [t for t in TRAIN if not (args.constant_only and t[0] == "7v")]
    X, y, rows = [], [], []
    for st, n, T in train:
        for dt in ("f64", "f32"):
            sw = Sweep(st, dt, *n, CONSTS[st], "mwd")
            r = timed_tune(sw, "exhaustive", T, args.budget)
            Xi, yi = C.records_from_log(sw, T, sw.tune_log())
            X += Xi
            y += yi
            for f, g in zip(Xi, yi):
                rows.append({"stencil": st, "dtype": dt, "grid": n, "T": T, "features": f, "glups": g})
            say("train %s %s %s: %d candidates, best %.1f GLUP/s, %.1f s" % (st, dt, n, r["measured"], r["glups"],
                                                                        r["seconds"]))
            sw.close()
    if args.log:
        with open(args.log, "w") as f:
            for r in rows:
                f.write(json.dumps(r) + "\n")
    model = C.CostModel(seed=0)
    t0 = time.perf_counter()
    losses = model.fit(X, y, steps=3000)
    t_fit = time.perf_counter() - t0
    pred = model.predict(X)
    fit_err = float(np.median(np.abs(np.log(pred) - np.log(np.asarray(y)))))
    say("model: %d records, loss %.4f -> %.4f, median |log error| %.3f, %.1f s" % (len(X), losses[0], losses[-1],
                                                                                  fit_err, t_fit))
    report = {"train_records": len(X), "train_loss_first": float(losses[0]), "train_loss_last": float(losses[-1]),
              "train_median_abs_log_error": fit_err, "train_seconds": t_fit,
              "train_problems": [[st, list(n), T] for st, n, T in train], "eval": []}
    for st, dt in EVAL:
        res = {"stencil": st, "dtype": dt, "grid": EVAL_GRID, "T": EVAL_T}
        sw = Sweep(st, dt, *EVAL_GRID, CONSTS[st], "mwd")
        res["exhaustive"] = timed_tune(sw, "exhaustive", EVAL_T, args.budget)
        res["hillclimb"] = timed_tune(sw, "hillclimb", EVAL_T, args.budget)
        res["model_top5"] = timed_tune(sw, "model", EVAL_T, args.budget, model.propose(sw, EVAL_T, 5))
        res["largest_tile"] = timed_tune(sw, "model", EVAL_T, args.budget, [largest_tile_pick(sw, EVAL_T)])
        # the four picks timed again together, interleaved, so that they are
        # compared under the same conditions
        methods = ("exhaustive", "hillclimb", "model_top5", "largest_tile")
        again = C.retime(sw, EVAL_T, [res[m]["params"] for m in methods])
        for i, m in enumerate(methods):
            res[m]["retimed"] = again[i]
        res["model_vs_exhaustive"] = res["model_top5"]["retimed"] / res["exhaustive"]["retimed"]
        res["model_vs_hillclimb"] = res["model_top5"]["retimed"] / res["hillclimb"]["retimed"]
        say("eval %s %s %s: exhaustive %.1f (%d, %.1f s), hill-climb %.1f (%d), model top-5 %.1f (%d, %.1f s), "
            "largest tile %.1f -> model/exhaustive %.3f"
            % (st, dt, EVAL_GRID, res["exhaustive"]["glups"], res["exhaustive"]["measured"],
               res["exhaustive"]["seconds"], res["hillclimb"]["glups"], res["hillclimb"]["measured"],
               res["model_top5"]["glups"], res["model_top5"]["measured"], res["model_top5"]["seconds"],
               res["largest_tile"]["glups"], res["model_vs_exhaustive"]))
        report["eval"].append(res)
        sw.close()
    txt = json.dumps(report)
    print(txt, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(txt + "\n")
    return 0


def summary(report_path, out_path, command):
    rep = json.loads(open(report_path).read())
    lines = ["# Learned cost model against the tuner", "",
             "Command: `%s`" % command, "",
             "Training: every feasible blocked candidate of %s, FP64 and FP32, measured by exhaustive search: "
             "%d records; loss %.4g -> %.4g (log GLUP/s squared), median absolute log error %.3f, %.1f s on the GPU."
             % (", ".join("%s %s T = %d" % (st, "x".join(str(v) for v in n), T)
                          for st, n, T in rep.get("train_problems", TRAIN)),
                rep["train_records"], rep["train_loss_first"], rep["train_loss_last"],
                rep["train_median_abs_log_error"], rep["train_seconds"]), "",
             "Evaluation on unseen problems: the GLUP/s of each search's pick, timed again after the "
             "searches with the four picks interleaved (three rounds, median), then the search's own best "
             "figure, the candidates it measured and its tuning seconds; pick = (diamond width, wavefront "
             "depth, x tile) waves along x x cells per lane, v = schedule / synchronisation variant.", "",
             "| problem | grid, T | exhaustive | hill climbing | model top-5 | largest tile that fits "
             "| model / exhaustive | model / hill climbing |", "|---|---|---|---|---|---|---|---|"]
    def pick(e):
        p = e.get("params", {})
        return "(%s)" % ", ".join(str(p.get(k, "")) for k in ("diamond_width", "wavefront_depth", "tile_x")
                                  if k in p) + ("" if "threads_x" not in p else
                                                " %dx%d" % (p["threads_x"] // 64, p["cells_per_lane"])) + \
            ("" if "variant" not in p else " v%d" % p["variant"])
    for r in rep["eval"]:
        def cell(k):
            e = r[k]
            head = "%.1f" % e["retimed"] if "retimed" in e else "-"
            return "%s; %.1f (%d, %.1f s) %s" % (head, e["glups"], e["measured"], e["seconds"], pick(e))
        lines.append("| %s %s | %s, %d | %s | %s | %s | %s | %.3f | %.3f |" % (
            r["stencil"], r["dtype"], "x".join(str(v) for v in r["grid"]), r["T"], cell("exhaustive"),
            cell("hillclimb"), cell("model_top5"), cell("largest_tile"), r["model_vs_exhaustive"],
            r.get("model_vs_hillclimb", r["model_top5"]["glups"] / r["hillclimb"]["glups"])))
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


def tgs(train_path, out_path, command):
    """Best rate per (problem, workgroup shape) from the training records
    (feature indices as in costmodel.features)."""
    rows = [json.loads(line) for line in open(train_path) if line.strip()]
    best = {}
    for r in rows:
        f = r["features"]
        prob = (r["stencil"], r["dtype"], tuple(r["grid"]), r["T"])
        dw, nf, tile = int(f[6]), int(f[7]), int(round(2 ** f[8]))
        wx, pairs, vx = int(f[11]), int(f[12]), int(f[13])
        variant = int(f[16]) + 2 * int(f[17])
        shape = (pairs * wx, wx, vx)
        cur = best.get((prob, shape))
        if cur is None or r["glups"] > cur[0]:
            best[(prob, shape)] = (r["glups"], dw, nf, tile, variant)
    lines = ["# Workgroup shape study (the paper's thread-group sizes, on the GPU)", "",
             "Command: `%s`" % command, "",
             "From the tuner's exhaustive measurements of the training problems (every feasible candidate, "
             "each timed on the problem's own T-step schedule): for each workgroup shape -- waves per tile "
             "(= row pairs Dw/2 x waves along x), waves along x, x cells per lane -- the best GLUP/s over "
             "diamond widths, wavefront depths, x tiles and schedule variants, and the candidate that reached "
             "it.  A wave is 64 lanes; a tile is one workgroup on one CU.", "",
             "| problem | waves per tile | waves along x | cells per lane | best GLUP/s | at (Dw, N_F, x tile, variant) |",
             "|---|---|---|---|---|---|"]
    for (prob, shape), (g, dw, nf, tile, variant) in sorted(best.items(), key=lambda kv: (kv[0][0], -kv[1][0])):
        st, dt, grid, T = prob
        lines.append("| %s %s %s, T = %d | %d | %d | %d | %.1f | (%d, %d, %d, %d) |"
                     % (st, dt, "x".join(str(v) for v in grid), T, shape[0], shape[1], shape[2], g, dw, nf, tile,
                        variant))
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "summary":
        summary(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
    elif len(sys.argv) > 1 and sys.argv[1] == "tgs":
        tgs(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
    else:
        sys.exit(main())
