"""The auto-tuner (paper, Section "Auto-tuning") on the GPU, through the C ABI:
exhaustive search measures every feasible candidate once and keeps the best;
the hill-climbing search measures a subset per thread shape; the model mode
measures exactly the candidates it is given, in order; a tuned plan still
computes the oracle's result bit for bit."""
import numpy as np
import pytest

from tests.gpu_util import inputs, oracle_run

pytestmark = pytest.mark.gpu


def plan(stencil="7c", dtype="f64", n=(160, 96, 64)):
    import paper_1510_04995_amd as P
    cc = [0.4, 0.1] if stencil == "7c" else [0.2, 0.05, 0.04, 0.03, 0.0133]
    return P.Sweep(stencil, dtype, *n, cc, "mwd")


def key(q):
    return (q["diamond_width"], q["tile_x"], q["threads_x"], q["cells_per_lane"])


def test_exhaustive_measures_every_candidate_and_keeps_the_best():
    sw = plan()
    cands = sw.candidates()
    best, rate = sw.tune("exhaustive", 32, 60.0)
    log = sw.tune_log()
    assert sorted(key(r["params"]) for r in log) == sorted(key(q) for q in cands)
    ok = [r for r in log if r["status"] == 0]
    assert ok and all(r["glups"] > 0 and r["seconds"] > 0 and r["steps"] > 0 for r in ok)
    top = max(ok, key=lambda r: r["glups"])
    assert rate == pytest.approx(top["glups"]) and key(best) == key(top["params"])
    assert key(sw.info()["params"]) == key(best)      # the plan keeps the winner
    sw.close()


def test_hillclimb_measures_a_subset():
    sw = plan(n=(256, 128, 64))
    n_all = len(sw.candidates())
    best, rate = sw.tune("hillclimb", 32, 60.0)
    log = sw.tune_log()
    assert 0 < len(log) <= n_all and rate > 0
    assert key(best) in {key(r["params"]) for r in log}
    sw.close()


def test_model_mode_measures_exactly_the_given_candidates():
    sw = plan()
    cands = sw.candidates()[:3]
    sw.set_candidates(cands)
    best, rate = sw.tune("model", 32, 30.0)
    log = sw.tune_log()
    assert [key(r["params"]) for r in log] == [key(q) for q in cands]
    assert rate > 0
    sw.set_candidates([])
    import paper_1510_04995_amd.girih as G
    with pytest.raises(G.GirihError) as e:
        sw.tune("model", 32, 30.0)
    assert e.value.code == G.E_UNSUPPORTED
    sw.close()


@pytest.mark.parametrize("stencil,dtype", [("7c", "f64"), ("25c", "f32")])
def test_tuned_plan_matches_the_oracle(stencil, dtype):
    import paper_1510_04995_amd as P
    from tests.gpu_util import run_gpu
    n = (150, 70, 40)
    sw = plan(stencil, dtype, n)
    best, _ = sw.tune("hillclimb", 16, 30.0)
    sw.close()
    u0, c, arr = inputs(stencil, *n, seed=12)
    got, _ = run_gpu(stencil, dtype, u0, c, arr, 9, algo="mwd", params=best)
    ref = oracle_run(stencil, u0, c, arr, 9, dtype)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("stencil,dtype,n,T", [("7c", "f64", (256, 256, 256), 64), ("25c", "f32", (192, 192, 192), 32)])
def test_tuned_rate_matches_timed_runs_of_the_problem(stencil, dtype, n, T):
    """The tuner times the problem's own T-step schedule (every diamond row,
    the clipped first and last included): its rate for a plan agrees with
    back-to-back girih_run calls of that plan timed with HIP events, within
    5 % (its own 3 % acceptance plus run-to-run noise)."""
    import torch
    from tests.gpu_util import upload
    sw = plan(stencil, dtype, n)
    q = sw.info()["params"]
    sw.set_candidates([q])
    _, rate = sw.tune("model", T, 30.0)
    u0, c, arr = inputs(stencil, *n, seed=13)
    b0 = upload(u0.astype(np.float64 if dtype == "f64" else np.float32))
    b1 = b0.clone()
    for _ in range(3):
        sw.run(b0, b1, T)
    times = []
    s = torch.cuda.current_stream()
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        sw.run(b0, b1, T)
        e1.record(s)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    run_rate = n[0] * n[1] * n[2] * T / sorted(times)[len(times) // 2] / 1e9
    print("%s %s: tuner %.1f GLUP/s, timed runs %.1f" % (stencil, dtype, rate, run_rate), flush=True)
    sw.close()
    assert abs(run_rate / rate - 1.0) < 0.05
