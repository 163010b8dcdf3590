"""Pins of the FP64 cost-model oracle (oracle/mlp.py) against facts that do
not come from the oracle itself: central finite differences of its own loss
(the gradient must be the derivative of what the forward pass computes), the
ReLU-linear regime against a plain chain of matrix products, the regime in
which every hidden unit is off, Adam's first step in closed form, and the
parameter count of the layer shapes."""
import numpy as np
import pytest

from oracle import mlp as M


def rand_params(rng, n_in, n_hidden, n_layers, scale=0.5):
    return rng.normal(0.0, scale, M.param_count(n_in, n_hidden, n_layers))


def test_param_count_matches_layer_shapes():
    assert M.param_count(16, 64, 3) == (64 * 16 + 64) + 2 * (64 * 64 + 64) + (64 + 1)
    assert M.param_count(3, 5, 1) == 3 * 5 + 5 + 5 + 1


@pytest.mark.parametrize("n_in,n_hidden,n_layers,n", [(5, 7, 3, 9), (16, 8, 1, 4), (3, 4, 2, 1)])
def test_gradient_matches_central_differences(n_in, n_hidden, n_layers, n):
    rng = np.random.default_rng(11)
    x = rng.normal(size=(n, n_in))
    t = rng.normal(size=n)
    p = rand_params(rng, n_in, n_hidden, n_layers)
    # keep every pre-activation away from the ReLU kink so the loss is smooth at p
    for _ in range(20):
        _, acts = M.forward(p, n_in, n_hidden, n_layers, x)
        layers = M.unpack(p, n_in, n_hidden, n_layers)
        zs = [acts[l] @ layers[l][0].T + layers[l][1] for l in range(n_layers)]
        if min(np.abs(z).min() for z in zs) > 1e-3:
            break
        p = rand_params(rng, n_in, n_hidden, n_layers)
    loss, g = M.loss_grad(p, n_in, n_hidden, n_layers, x, t)
    h = 1e-6
    num = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = M.loss_grad(p + e, n_in, n_hidden, n_layers, x, t)
        lm, _ = M.loss_grad(p - e, n_in, n_hidden, n_layers, x, t)
        num[i] = (lp - lm) / (2 * h)
    assert np.linalg.norm(g - num) <= 1e-6 * max(1.0, np.linalg.norm(num))


def test_linear_regime_equals_matrix_chain():
    # positive inputs, weights and biases: every ReLU passes its input, so the
    # network is the affine map W_L ... W_1 x + (propagated biases)
    rng = np.random.default_rng(5)
    n_in, n_hidden, n_layers, n = 6, 5, 3, 7
    p = np.abs(rand_params(rng, n_in, n_hidden, n_layers)) + 0.01
    x = np.abs(rng.normal(size=(n, n_in))) + 0.01
    y, _ = M.forward(p, n_in, n_hidden, n_layers, x)
    layers = M.unpack(p, n_in, n_hidden, n_layers)
    A = np.linalg.multi_dot([W for W, _ in layers[::-1]])        # (1, n_in)
    c = np.zeros(n_in)
    for W, b in layers:
        c = W @ c + b
    expect = (x @ A.T)[:, 0] + c[0]
    assert np.allclose(y, expect, rtol=1e-12, atol=1e-12)


def test_dead_hidden_layer_outputs_the_bias():
    rng = np.random.default_rng(6)
    n_in, n_hidden, n_layers = 4, 6, 2
    p = rand_params(rng, n_in, n_hidden, n_layers)
    layers = M.unpack(p, n_in, n_hidden, n_layers)
    # first layer: negative weights and biases on positive inputs -> all units off
    o = 0
    fo, fi = M.layer_shapes(n_in, n_hidden, n_layers)[0]
    p[o:o + fo * fi] = -np.abs(p[o:o + fo * fi]) - 0.1
    p[o + fo * fi:o + fo * fi + fo] = -0.5
    x = np.abs(rng.normal(size=(5, n_in)))
    y, _ = M.forward(p, n_in, n_hidden, n_layers, x)
    layers = M.unpack(p, n_in, n_hidden, n_layers)
    # second hidden layer sees zeros: relu(b1); output = W_out relu(b1) + b_out
    W1, b1 = layers[1]
    Wo, bo = layers[2]
    expect = Wo @ np.maximum(b1, 0) + bo
    assert np.allclose(y, expect[0], rtol=0, atol=1e-15)
    # and no gradient reaches the first layer's weights
    _, g = M.loss_grad(p, n_in, n_hidden, n_layers, x, np.zeros(5))
    assert np.all(g[:fo * fi + fo] == 0)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(7)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    p1, m1, v1 = M.adam(p, g, np.zeros(50), np.zeros(50), lr, b1, b2, eps, 1)
    # bias-corrected moments after one step are g and g^2
    assert np.allclose(m1, (1 - b1) * g, rtol=1e-15, atol=0)
    assert np.allclose(v1, (1 - b2) * g * g, rtol=1e-15, atol=0)
    assert np.allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)


def test_zero_error_has_zero_loss_and_gradient():
    rng = np.random.default_rng(8)
    n_in, n_hidden, n_layers = 3, 4, 2
    p = rand_params(rng, n_in, n_hidden, n_layers)
    x = rng.normal(size=(6, n_in))
    y, _ = M.forward(p, n_in, n_hidden, n_layers, x)
    loss, g = M.loss_grad(p, n_in, n_hidden, n_layers, x, y)
    assert loss == 0.0 and np.all(g == 0)


def test_plant_wrong_sign_is_caught():
    # a gradient with a flipped sign (a plausible mistake) fails the difference check
    rng = np.random.default_rng(9)
    n_in, n_hidden, n_layers = 3, 4, 1
    p = rand_params(rng, n_in, n_hidden, n_layers)
    x = rng.normal(size=(5, n_in))
    t = rng.normal(size=5)
    _, g = M.loss_grad(p, n_in, n_hidden, n_layers, x, t)
    h = 1e-6
    e = np.zeros_like(p)
    e[-1] = h                                # the output bias
    num = (M.loss_grad(p + e, n_in, n_hidden, n_layers, x, t)[0] - M.loss_grad(p - e, n_in, n_hidden, n_layers, x, t)[0]) / (2 * h)
    assert abs(g[-1] - num) < 1e-6 and abs(-g[-1] - num) > 1e-3


def test_zero_network_loss_is_the_mean_of_squared_targets():
    """With every parameter zero the network outputs 0, so the loss is the
    mean of t^2 (the 1/n of the mean squared error, not the sum) and the only
    nonzero gradient entry is the output bias's, 2 * mean(0 - t)."""
    rng = np.random.default_rng(3)
    n_in, n_hidden, n_layers, n = 4, 6, 3, 11
    p = np.zeros(M.param_count(n_in, n_hidden, n_layers))
    x = rng.normal(size=(n, n_in))
    t = rng.normal(size=n)
    loss, g = M.loss_grad(p, n_in, n_hidden, n_layers, x, t)
    assert loss == pytest.approx(float(np.dot(t, t)) / n, rel=1e-15)
    assert g[-1] == pytest.approx(-2.0 * t.sum() / n, rel=1e-15)
    assert np.all(g[:-1] == 0)
