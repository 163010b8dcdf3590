"""GPU checks of the cost model's HIP kernels (girih_mlp_*) against the FP64
oracle (oracle/mlp.py), and of what the trained model gains the tuner.

Tolerances: the kernels compute in FP32 with sums of at most 64 terms in a
fixed order; relative errors of a few FP32 ulps times the term count are
expected (forward 1e-5, gradient 1e-4 in relative L2, Adam 1e-6)."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N_IN, N_H, N_L = 16, 64, 3


def dev():
    import torch
    return torch, torch.device("cuda:0")


def test_forward_matches_oracle():
    from oracle import mlp as M
    from paper_1510_04995_amd import costmodel as C, girih as G
    torch, d = dev()
    p = C.he_uniform(N_IN, N_H, N_L, seed=3)
    rng = np.random.default_rng(1)
    x = rng.normal(size=(37, N_IN)).astype(np.float32)
    ref, _ = M.forward(p.astype(np.float64), N_IN, N_H, N_L, x.astype(np.float64))
    pg, xg = torch.from_numpy(p).to(d), torch.from_numpy(x).to(d)
    y = torch.empty(37, dtype=torch.float32, device=d)
    wl = G.girih_mlp_work_count(N_IN, N_H, N_L, 37)
    w = torch.empty(wl, dtype=torch.float32, device=d)
    G.girih_mlp_forward(pg.data_ptr(), N_IN, N_H, N_L, xg.data_ptr(), 37, y.data_ptr(), w.data_ptr(), wl,
                        torch.cuda.current_stream().cuda_stream)
    got = y.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)


@pytest.mark.parametrize("n", [1, 5, 300])
def test_loss_and_gradient_match_oracle(n):
    from oracle import mlp as M
    from paper_1510_04995_amd import costmodel as C, girih as G
    torch, d = dev()
    p = C.he_uniform(N_IN, N_H, N_L, seed=4)
    rng = np.random.default_rng(n)
    x = rng.normal(size=(n, N_IN)).astype(np.float32)
    t = rng.normal(size=n).astype(np.float32)
    loss_ref, g_ref = M.loss_grad(p.astype(np.float64), N_IN, N_H, N_L, x.astype(np.float64), t.astype(np.float64))
    pg, xg, tg = (torch.from_numpy(a).to(d) for a in (p, x, t))
    loss = torch.empty(1, dtype=torch.float32, device=d)
    grad = torch.empty(p.size, dtype=torch.float32, device=d)
    wl = G.girih_mlp_work_count(N_IN, N_H, N_L, n)
    w = torch.empty(wl, dtype=torch.float32, device=d)
    G.girih_mlp_loss_grad(pg.data_ptr(), N_IN, N_H, N_L, xg.data_ptr(), tg.data_ptr(), n, loss.data_ptr(),
                          grad.data_ptr(), w.data_ptr(), wl, torch.cuda.current_stream().cuda_stream)
    g = grad.cpu().numpy().astype(np.float64)
    assert abs(float(loss.cpu()) - loss_ref) <= 1e-5 * loss_ref
    assert np.linalg.norm(g - g_ref) <= 1e-4 * np.linalg.norm(g_ref)


def test_adam_step_matches_oracle():
    from oracle import mlp as M
    from paper_1510_04995_amd import girih as G
    torch, d = dev()
    rng = np.random.default_rng(2)
    n = 1000
    p, g = rng.normal(size=n).astype(np.float32), rng.normal(size=n).astype(np.float32)
    m, v = (rng.normal(size=n) * 0.1).astype(np.float32), np.abs(rng.normal(size=n) * 0.01).astype(np.float32)
    for step in (1, 7):
        pr, mr, vr = M.adam(p, g, m, v, 1e-3, 0.9, 0.999, 1e-8, step)
        pg, gg, mg, vg = (torch.from_numpy(a.copy()).to(d) for a in (p, g, m, v))
        G.girih_mlp_adam(pg.data_ptr(), gg.data_ptr(), mg.data_ptr(), vg.data_ptr(), n, 1e-3, 0.9, 0.999, 1e-8, step,
                         torch.cuda.current_stream().cuda_stream)
        for got, ref in ((pg, pr), (mg, mr), (vg, vr)):
            a = got.cpu().numpy().astype(np.float64)
            assert np.max(np.abs(a - ref)) <= 1e-6 * max(1.0, np.max(np.abs(ref)))


def test_training_fits_a_smooth_target():
    from paper_1510_04995_amd import costmodel as C
    rng = np.random.default_rng(5)
    X = rng.normal(size=(400, C.N_FEATURES))
    w = rng.normal(size=C.N_FEATURES) * 0.3
    y = np.exp(2.0 + X @ w + 0.1 * np.sin(X[:, 0]))
    m = C.CostModel(seed=1)
    losses = m.fit(X, y, steps=1500, lr=3e-3)
    assert losses[-1] < 0.05 * losses[0]
    pred = m.predict(X[:50])
    assert np.median(np.abs(np.log(pred) - np.log(y[:50]))) < 0.1


def test_model_proposals_reach_exhaustive_with_fewer_measurements():
    """Train on the tuner's measurements of three small constant-coefficient
    problems, then tune an unseen problem -- the 7-point variable-coefficient
    stencil, FP64 and FP32: the model's top-5 must reach 90 % of exhaustive
    search's best while measuring fewer candidates than exhaustive search and
    than the paper's hill-climbing tuner, at a rate within 10 % of hill
    climbing's; the picks are compared re-timed together."""
    import paper_1510_04995_amd as P
    from paper_1510_04995_amd import costmodel as C
    X, y = [], []
    for st, dt, n, T in (("7c", "f64", (96, 96, 96), 32), ("7c", "f32", (128, 128, 64), 32),
                         ("25c", "f64", (96, 96, 96), 16)):
        cc = [0.4, 0.1] if st == "7c" else [0.2, 0.05, 0.04, 0.03, 0.0133]
        sw = P.Sweep(st, dt, *n, cc, "mwd")
        sw.tune("exhaustive", T, 20.0)
        Xi, yi = C.records_from_log(sw, T, sw.tune_log())
        X += Xi
        y += yi
        sw.close()
    assert len(X) >= 30
    model = C.CostModel(seed=0)
    losses = model.fit(X, y, steps=2000)
    assert losses[-1] < losses[0]
    nx, ny, nz, T = 128, 192, 256, 32
    for dt in ("f64", "f32"):
        ex = P.Sweep("7v", dt, nx, ny, nz, None, "mwd")
        t0 = time.perf_counter()
        p_exh, best_exh = ex.tune("exhaustive", T, 60.0)
        t_exh = time.perf_counter() - t0
        n_exh = len(ex.tune_log())
        t0 = time.perf_counter()
        p_mlp, best_mlp, n_mlp = C.tune_with_model(ex, model, T, k=5)
        t_mlp = time.perf_counter() - t0
        hc = P.Sweep("7v", dt, nx, ny, nz, None, "mwd")
        p_hc, best_hc = hc.tune("hillclimb", T, 60.0)
        n_hc = len(hc.tune_log())
        # the three picks timed again together (interleaved), so that they are
        # compared under the same conditions
        again = C.retime(ex, T, [p_exh, p_hc, p_mlp])
        print("7v %s: exhaustive %.1f GLUP/s (%d measured, %.1f s); model top-5 %.1f (%d, %.1f s); "
              "hill-climb %.1f (%d); re-timed %.1f / %.1f / %.1f"
              % (dt, best_exh, n_exh, t_exh, best_mlp, n_mlp, t_mlp, best_hc, n_hc, again[0], again[1], again[2]),
              flush=True)
        assert n_mlp <= 5 < n_exh
        assert p_mlp == p_exh or again[2] >= 0.9 * again[0]
        # fewer measurements than the paper's tuner, at a rate within the same
        # 10 % (on this small grid the best candidates lie within a few per cent
        # of each other, about the spread of repeated measurements)
        assert n_mlp < n_hc and (p_mlp == p_hc or again[2] >= 0.9 * again[1])
        ex.close()
        hc.close()
