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
