"""Plain FP64 reference of the tuner's cost model — TEST INFRASTRUCTURE ONLY.

Only the test-suite uses this module; the product computes the network with
the HIP kernels of ``libgirih.so`` (``girih_mlp_*``).  It shares no code with
them.

What it computes (the definitions, written out):

* network: ``n_in`` inputs -> ``n_layers`` hidden layers of ``n_hidden`` units,
  ``a = relu(W a_prev + b)`` -> one linear output ``y = W a + b``;
* parameters: one flat array, layer by layer (first hidden layer first, the
  output layer last), each ``W`` (fan_out x fan_in, row-major) then ``b``;
* loss: mean squared error ``(1/n) sum_i (y_i - t_i)^2``;
* gradient: back-propagation of that loss (the chain rule, layer by layer);
* Adam (Kingma and Ba, 2015, Algorithm 1): ``m = b1 m + (1-b1) g``,
  ``v = b2 v + (1-b2) g^2``, ``p -= lr * (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps)``.

Parity status: pinned by ``tests/test_mlp_oracle.py`` (central finite
differences, the linear regime against a plain matrix product, the dead-ReLU
regime, Adam's first step in closed form).
"""
import numpy as np


def layer_shapes(n_in, n_hidden, n_layers):
    """[(fan_out, fan_in)] of every layer, output layer last."""
    shapes = [(n_hidden, n_in)]
    shapes += [(n_hidden, n_hidden)] * (n_layers - 1)
    shapes.append((1, n_hidden))
    return shapes


def param_count(n_in, n_hidden, n_layers):
    return sum(fo * fi + fo for fo, fi in layer_shapes(n_in, n_hidden, n_layers))


def unpack(params, n_in, n_hidden, n_layers):
    """[(W, b)] views of the flat parameter array (float64 copies)."""
    p = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for fo, fi in layer_shapes(n_in, n_hidden, n_layers):
        W = p[o:o + fo * fi].reshape(fo, fi)
        o += fo * fi
        b = p[o:o + fo]
        o += fo
        out.append((W, b))
    assert o == p.size, "parameter array has the wrong length"
    return out


def forward(params, n_in, n_hidden, n_layers, x):
    """Network output (n,) and the list of layer inputs (x, then each hidden activation)."""
    layers = unpack(params, n_in, n_hidden, n_layers)
    a = np.asarray(x, dtype=np.float64)
    acts = [a]
    for l, (W, b) in enumerate(layers):
        z = a @ W.T + b
        a = np.maximum(z, 0.0) if l < len(layers) - 1 else z
        acts.append(a)
    return acts[-1][:, 0], acts[:-1]


def loss_grad(params, n_in, n_hidden, n_layers, x, t):
    """(loss, flat gradient) of the mean squared error."""
    layers = unpack(params, n_in, n_hidden, n_layers)
    y, acts = forward(params, n_in, n_hidden, n_layers, x)
    t = np.asarray(t, dtype=np.float64)
    n = y.size
    err = y - t
    loss = float(np.sum(err * err) / n)
    delta = (2.0 * err / n)[:, None]          # dL/dz of the output layer, (n, 1)
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        a_in = acts[l]
        grads[l] = (delta.T @ a_in, delta.sum(axis=0))
        if l > 0:
            delta = (delta @ W) * (a_in > 0)    # back through W, then through the ReLU of layer l-1
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam(p, g, m, v, lr, b1, b2, eps, step):
    """One Adam step; returns (p, m, v) as new float64 arrays."""
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
