"""Pins of the oracle's second-order-in-time 25-point stencil (Listing 3 as
printed: u^{t+1} = (2 u^t - u^{t-1}) + C * L(u^t), L the radius-4 star with
constants c0..c4), against facts the mathematics fixes (no GPU):

* C = 0 leaves the field unchanged bit for bit (2u - u = u);
* a sine mode with constant C follows the three-term recurrence
  a_{t+1} = (2 + C*lambda) a_t - a_{t-1} inside the light cone;
* exact rational evaluation on an 8^3 grid (independent code below);
* the scheme is time-reversible: swapping the two buffers after T steps and
  running T more steps returns to the start (within rounding);
* an impulse spreads R cells per step and no further.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import sweep as osw
from workloads import field_and_coefs
from workloads.grids import laplacian8_weights

R = 4


def run(u0, T, consts, C, prev=None, dtype=np.float64):
    b0 = np.ascontiguousarray(u0.astype(dtype))
    b1 = np.ascontiguousarray((u0 if prev is None else prev).astype(dtype))
    idx = osw.sweep("25l", b0, b1, T, np.asarray(consts, dtype=dtype), [np.ascontiguousarray(C.astype(dtype))])
    return (b0, b1)[idx], (b0, b1)[1 - idx]


def sine_field(nx, ny, nz, p, q, r):
    z = np.sin(r * math.pi * np.arange(1, nz + 1) / (nz + 1))
    y = np.sin(q * math.pi * np.arange(1, ny + 1) / (ny + 1))
    x = np.sin(p * math.pi * np.arange(1, nx + 1) / (nx + 1))
    u = np.zeros((nz + 2 * R, ny + 2 * R, nx + 2 * R))
    u[R:R + nz, R:R + ny, R:R + nx] = z[:, None, None] * y[None, :, None] * x[None, None, :]
    return u


def test_zero_courant_number_keeps_the_field_bitwise():
    u0, c, arr = field_and_coefs("25l", 13, 11, 12, seed=2)
    out, prev = run(u0, 7, c, np.zeros_like(arr[0]))
    assert np.array_equal(out, u0) and np.array_equal(prev, u0)


def test_sine_mode_follows_the_three_term_recurrence():
    nx, ny, nz, T = 45, 41, 47, 3
    p, q, r = 2, 3, 1
    u0 = sine_field(nx, ny, nz, p, q, r)
    c = laplacian8_weights()
    cc = 0.07
    C = np.full_like(u0, cc)
    out, _ = run(u0, T, c, C)
    th = [p * math.pi / (nx + 1), q * math.pi / (ny + 1), r * math.pi / (nz + 1)]
    lam = c[0] + 2 * sum(c[m] * sum(math.cos(m * t) for t in th) for m in range(1, 5))
    a_prev, a = 1.0, 1.0                     # u^{-1} = u^0
    for _ in range(T):
        a_prev, a = a, (2 + cc * lam) * a - a_prev
    reach = R * T
    sl = tuple(slice(R + reach, R + n - reach) for n in (nz, ny, nx))
    assert out[sl].size > 1000
    assert np.max(np.abs(out[sl] - a * u0[sl])) <= 1e-13 * np.max(np.abs(u0[sl]))
    # the mode really changed (a is not 1), so the recurrence is exercised
    assert abs(a - 1.0) > 1e-3


def exact_leapfrog(u0, prev, T, consts, C):
    """The sweep in rational arithmetic, written from the listing."""
    F = np.vectorize(Fraction, otypes=[object])
    cur, old = F(u0), F(prev)
    c = [Fraction(float(v)) for v in consts]
    Cq = F(C)
    nzp, nyp, nxp = u0.shape
    nz, ny, nx = nzp - 2 * R, nyp - 2 * R, nxp - 2 * R
    inner = (slice(R, R + nz), slice(R, R + ny), slice(R, R + nx))

    def at(a, dz, dy, dx):
        return a[R + dz:R + dz + nz, R + dy:R + dy + ny, R + dx:R + dx + nx]

    for _ in range(T):
        b = c[0] * at(cur, 0, 0, 0)
        for r in range(1, R + 1):
            s = (at(cur, 0, 0, r) + at(cur, 0, 0, -r) + at(cur, 0, r, 0) + at(cur, 0, -r, 0)
                 + at(cur, r, 0, 0) + at(cur, -r, 0, 0))
            b = b + c[r] * s
        new = old.copy()
        new[inner] = 2 * at(cur, 0, 0, 0) - at(old, 0, 0, 0) + Cq[inner] * b
        old, cur = cur, new
    return np.vectorize(float, otypes=[np.float64])(cur)


@pytest.mark.parametrize("seed", [4, 9])
def test_exact_rational_8cubed(seed):
    u0, c, arr = field_and_coefs("25l", 8, 8, 8, seed=seed)
    rng = np.random.default_rng(seed)
    prev = u0.copy()
    prev[R:-R, R:-R, R:-R] = rng.random((8, 8, 8))      # a nonzero initial velocity
    T = 3
    exact = exact_leapfrog(u0, prev, T, c, arr[0])
    out, _ = run(u0, T, c, arr[0], prev)
    scale = np.max(np.abs(exact))
    assert np.max(np.abs(out - exact)) <= T * 32 * 2.0 ** -53 * 20 * scale
    assert np.linalg.norm(out - exact) <= 1e-13 * np.linalg.norm(exact)
    out32, _ = run(u0, T, c, arr[0], prev, dtype=np.float32)
    assert np.max(np.abs(out32 - exact)) <= (T + 1) * 32 * 2.0 ** -24 * 20 * scale


def test_time_reversal_returns_to_the_start():
    u0, c, arr = field_and_coefs("25l", 20, 18, 19, seed=6)
    T = 8
    out, prev = run(u0, T, c, arr[0])
    # the state after T steps is (u^{T-1}, u^T); running the same scheme from
    # (current = u^{T-1}, previous = u^T) walks back to (u^0, u^{-1}) = (u^0, u^0)
    back, back_prev = run(prev, T, c, arr[0], prev=out)
    assert np.max(np.abs(back - u0)) <= 1e-12
    assert np.max(np.abs(back_prev - u0)) <= 1e-12
    assert np.max(np.abs(out - u0)) > 1e-3          # the forward run did move


def test_impulse_spreads_R_cells_per_step():
    n, T = 33, 3
    u0 = np.zeros((n + 2 * R,) * 3)
    m = R + n // 2
    u0[m, m, m] = 1.0
    C = np.full_like(u0, 0.05)
    out, _ = run(u0, T, laplacian8_weights(), C)
    nz = np.argwhere(out != 0)
    dist = np.abs(nz - m).sum(axis=1)
    # star stencil: the support is the union of axis moves of length <= R per
    # step, so the L1 distance grows by at most R per step and the axis tips
    # at distance R*T are reached
    assert dist.max() == R * T
    assert out[m, m, m + R * T] != 0 and out[m, m, m + R * T + 1] == 0
