"""The measurement tools' arithmetic on synthetic counter files (CPU only):
bytes per update from FETCH_SIZE / WRITE_SIZE scaled by a copy of known size,
in-core utilisation from SQ counters, and the throughput table."""
import csv
import json

import pytest

from paper_1510_04995_amd import dw_sweep, energy, profsum, suite


def _write_counters(path, rows):
    keys = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=keys)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(keys, r)))


def test_dw_sweep_bytes_per_update(tmp_path):
    # one naive case (2 launches) and one blocked case (3 launches) on 4x4x4, T = 2;
    # the counter reads half of the copy's bytes for FETCH_SIZE (factor 2)
    cases = [{"stencil": "7c", "dtype": "f64", "grid": [4, 4, 4], "T": 2, "algo": "naive",
              "params": {"diamond_width": 0, "tile_x": 64, "threads_x": 64, "cells_per_lane": 1},
              "model_bytes_per_lup": 16.0, "launches": 2},
             {"stencil": "7c", "dtype": "f64", "grid": [4, 4, 4], "T": 2, "algo": "mwd",
              "params": {"diamond_width": 4, "tile_x": 4, "threads_x": 128, "cells_per_lane": 2},
              "model_bytes_per_lup": 9.0, "launches": 3}]
    log = tmp_path / "run.log"
    log.write_text("\n".join(json.dumps(c) for c in cases) + "\n")
    lups = 4 * 4 * 4 * 2
    fetch, write = [], []
    d = 0
    for name, kib in (("naive_step_kernel<x>", 0.5), ("naive_step_kernel<x>", 0.5),
                      ("mwd_row_kernel<y>", 0.25), ("mwd_row_kernel<y>", 0.25), ("mwd_row_kernel<y>", 0.25),
                      ("__amd_rocclr_copyBuffer", 512.0)):
        d += 1
        fetch.append((d, name, "FETCH_SIZE", kib, 0, 1))
        write.append((d, name, "WRITE_SIZE", 2 * kib, 0, 1))
    _write_counters(tmp_path / "f.csv", fetch)
    _write_counters(tmp_path / "w.csv", write)
    out = tmp_path / "out.md"
    dw_sweep.summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(log), "1", str(out), "cmd")
    text = out.read_text()
    # naive: fetch 1 KiB x 2 + write 2 KiB x 1 = 4 KiB over 128 updates = 32 B
    assert "| 7c f64 | naive | - | 64 | 64 | 2 | %.2f | 16.00 |" % (4096.0 / lups) in text
    # blocked: fetch 0.75 KiB x 2 + write 1.5 KiB = 3 KiB
    assert "| 7c f64 | mwd | 4 | 4 | 128 | 3 | %.2f | 9.00 |" % (3072.0 / lups) in text


def test_dw_sweep_rejects_a_dispatch_count_mismatch(tmp_path):
    case = {"stencil": "7c", "dtype": "f64", "grid": [4, 4, 4], "T": 2, "algo": "naive",
            "params": {"diamond_width": 0, "tile_x": 64, "threads_x": 64, "cells_per_lane": 1},
            "model_bytes_per_lup": 16.0, "launches": 2}
    (tmp_path / "run.log").write_text(json.dumps(case) + "\n")
    rows = [(1, "naive_step_kernel", c, 1.0, 0, 1) for c in ("FETCH_SIZE",)] + [
        (2, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 4.0, 0, 1)]
    _write_counters(tmp_path / "f.csv", rows)
    _write_counters(tmp_path / "w.csv", [(r[0], r[1], "WRITE_SIZE", r[3], 0, 1) for r in rows])
    with pytest.raises(SystemExit):
        dw_sweep.summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "run.log"), "1",
                         str(tmp_path / "o.md"), "cmd")


def _bench_line(tmp_path):
    b = {"metric": "m", "value": 500.0, "dtype": "f64",
         "config": {"workload": "w", "kernel_source_hash": "h",
                    "params": {"diamond_width": 12, "tile_x": 106, "threads_x": 128, "cells_per_lane": 1}},
         "roofline": {"frac": 0.4, "bytes_per_lup_alg": 5.33, "launches": 12, "avg_launch_ms": 1.0}}
    p = tmp_path / "bench.json"
    p.write_text(json.dumps(b) + "\n")
    return p


def test_core_utilisation(tmp_path):
    name = "void girih::mwd_row_kernel<girih::Stencil7C, double, 12, 1, 2, 0>(x)"
    other = "void girih::mwd_row_kernel<girih::Stencil7C, float, 12, 1, 2, 0>(x)"
    ns = 1.0e6                      # 1 ms
    cyc = 2.0e6                     # 2 GHz
    a = [(1, name, "GRBM_GUI_ACTIVE", 8 * cyc, 0, ns), (1, name, "SQ_WAVES", 1000, 0, ns),
         (1, name, "SQ_INSTS_VALU", 4.0e8, 0, ns), (1, name, "SQ_ACTIVE_INST_VALU", 0.25 * 1024 * cyc / 4, 0, ns),
         (1, name, "SQ_INSTS_VALU_ADD_F64", 1.0e8, 0, ns), (1, name, "SQ_INSTS_VALU_MUL_F64", 1.0e8, 0, ns),
         (1, name, "SQ_INSTS_LDS", 5.0e7, 0, ns), (1, name, "SQ_LDS_IDX_ACTIVE", 0.5 * 256 * cyc, 0, ns),
         (1, name, "SQ_LDS_BANK_CONFLICT", 0, 0, ns),
         (2, other, "SQ_WAVES", 99, 0, ns)]
    b = [(1, name, "SQ_INSTS_LDS_LOAD_BANDWIDTH", 256 * cyc * 32 / 64, 0, ns),
         (1, name, "SQ_INSTS_LDS_STORE_BANDWIDTH", 256 * cyc * 32 / 64, 0, ns),
         (1, name, "SQ_INSTS_SALU", 1.0e7, 0, ns), (1, name, "GRBM_GUI_ACTIVE", 8 * cyc, 0, ns)]
    _write_counters(tmp_path / "a.csv", a)
    _write_counters(tmp_path / "b.csv", b)
    out = tmp_path / "core.md"
    profsum.core(str(tmp_path / "a.csv"), str(tmp_path / "b.csv"), str(_bench_line(tmp_path)), str(out), "cmd")
    t = out.read_text()
    assert "| shader clock (GRBM_GUI_ACTIVE / duration) | 2.00 GHz |" in t
    assert "| VALU busy, all 1024 SIMDs (4 x SQ_ACTIVE_INST_VALU / SIMD cycles) | 25.0 % |" in t
    assert "| waves per launch | 1000 |" in t
    # 64 lanes x 2e8 FP64 instructions in 1 ms = 12.8 TFLOP/s
    assert "12.80 TFLOP/s" in t
    assert "LDS busy, all 256 CUs (SQ_LDS_IDX_ACTIVE / CU cycles) | 50.0 %" in t
    assert "64.0 of 128" in t


def test_suite_table(tmp_path):
    recs = [{"workload": "device-copy", "bytes": 2.0, "seconds": 1.0, "gb_per_s": 4800.0},
            {"workload": "w", "stencil": "7c", "grid": [8, 8, 8], "T": 2, "dtype": "f64", "algo": "naive",
             "glups": 200.0, "seconds": 1.0, "model_bytes_per_lup": 16.0,
             "params": {"diamond_width": 0, "tile_x": 64, "threads_x": 64, "cells_per_lane": 1}},
            {"workload": "w", "stencil": "7c", "grid": [8, 8, 8], "T": 2, "dtype": "f64", "algo": "mwd",
             "glups": 500.0, "seconds": 1.0, "model_bytes_per_lup": 6.0, "bitwise_diff_vs_naive_f64": 0,
             "params": {"diamond_width": 12, "tile_x": 106, "threads_x": 128, "cells_per_lane": 1}},
            {"workload": "w", "stencil": "25v", "grid": [8, 8, 8], "T": 2, "dtype": "f32", "algo": "naive",
             "glups": 60.0, "seconds": 1.0, "model_bytes_per_lup": 60.0, "rel_l2_vs_f64": 1e-7,
             "max_abs_vs_f64": 2e-7,
             "params": {"diamond_width": 0, "tile_x": 64, "threads_x": 64, "cells_per_lane": 1}}]
    log = tmp_path / "s.log"
    log.write_text("\n".join(json.dumps(r) for r in recs) + "\n")
    out = tmp_path / "s.md"
    suite.summary(str(log), str(out), "cmd")
    t = out.read_text()
    assert "copy runs at 4800 GB/s" in t
    assert "| w | f64 | naive | 200.0 | 500 | 16.00 | - | reference |" in t
    assert "| w | f64 | mwd | 500.0 | 500 | 6.00 | 12, 106, 128, 1 | 0 differ |" in t
    # 25v FP32: (2 + 13) x 4 B per update at 8 TB/s = 133 GLUP/s
    assert "| w | f32 | naive | 60.0 | 133 | 60.00 | - | 1.00e-07 / 2.00e-07 |" in t


def test_energy_table(tmp_path):
    recs = [{"case": "idle", "power_w": 250.0, "samples": 5},
            {"case": "7c f64 mwd", "stencil": "7c", "dtype": "f64", "algo": "mwd", "grid": [512, 512, 512], "T": 64,
             "runs": 10, "glups": 500.0, "power_w": 1000.0, "samples": 20, "nj_per_lup": 2.0, "params": {}},
            {"case": "7c f64 naive", "stencil": "7c", "dtype": "f64", "algo": "naive", "grid": [512, 512, 512],
             "T": 64, "runs": 10, "glups": 250.0, "power_w": None, "samples": 0, "nj_per_lup": None, "params": {}}]
    log = tmp_path / "e.log"
    log.write_text("\n".join(json.dumps(r) for r in recs) + "\n")
    out = tmp_path / "e.md"
    energy.summary(str(log), str(out), "cmd")
    t = out.read_text()
    assert "Idle power before the runs: 250 W." in t
    assert "| 7c f64 mwd | 512x512x512, 64 | 500.0 | 1000 | 20 | 2.000 |" in t
    assert "| 7c f64 naive | 512x512x512, 64 | 250.0 | n/a | 0 | n/a |" in t


def test_socket_power_parser(monkeypatch):
    class R:
        stdout = json.dumps({"gpu_data": [{"gpu": 0, "power": {"socket_power": {"value": 262, "unit": "W"}}}]})
    monkeypatch.setattr(energy.subprocess, "run", lambda *a, **k: R())
    assert energy.socket_power_w() == 262.0
    R.stdout = "not json"
    assert energy.socket_power_w() is None


def test_tune_study_table(tmp_path):
    from paper_1510_04995_amd import tune_study

    def e(g, m, t):
        return {"glups": g, "measured": m, "seconds": t, "params": {}}
    rep = {"train_records": 176, "train_loss_first": 26.9, "train_loss_last": 0.0009,
           "train_median_abs_log_error": 0.007, "train_seconds": 3.5,
           "eval": [{"stencil": "7c", "dtype": "f64", "grid": [256, 512, 1024], "T": 64,
                     "exhaustive": e(400.0, 28, 6.5), "hillclimb": e(399.0, 15, 3.0),
                     "model_top5": e(398.0, 5, 1.2), "largest_tile": e(304.2, 1, 0.3),
                     "model_vs_exhaustive": 0.995}]}
    p = tmp_path / "r.json"
    p.write_text(json.dumps(rep))
    out = tmp_path / "t.md"
    tune_study.summary(str(p), str(out), "cmd")
    t = out.read_text()
    assert "176 records; loss 26.9 -> 0.0009" in t
    assert ("| 7c f64 | 256x512x1024, 64 | -; 400.0 (28, 6.5 s) () | -; 399.0 (15, 3.0 s) () | -; 398.0 (5, 1.2 s) () "
            "| -; 304.2 (1, 0.3 s) () | 0.995 | 0.997 |") in t
