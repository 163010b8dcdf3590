"""Pins of the CPU oracle against facts fixed by the mathematics (no GPU).

Each test is chosen so that a plausible slip in the oracle — a dropped term, a
wrong sign or radius, a transposed axis, a wrong buffer swap — fails at least
one of them:

* sine eigenmode of the 7-point operator with zero Dirichlet halo: exact
  closed-form decay lambda^T (catches wrong weights, wrong axis sizes);
* the same mode for the radius-4 star, inside the light cone;
* constant field with weights summing to one is preserved;
* exact rational evaluation on 8^3 grids (all four stencils), independent
  term-table code in ``exact_dyadic.py``;
* mirror symmetry (bitwise) for the constant-coefficient stencils;
* light cone of a unit impulse (support exactly as the radius predicts);
* linearity, and time-splitting run(T1);run(T2) == run(T1+T2) bitwise;
* variable-coefficient stencils with constant coefficient arrays reduce to the
  constant-coefficient ones.
"""
import math
import os

import numpy as np
import pytest

from oracle import sweep as osw
from workloads import field_and_coefs
from tests.exact_dyadic import exact_sweep, to_float

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def run(stencil, u0, T, consts=None, arrays=None, dtype=np.float64):
    b0 = np.ascontiguousarray(u0.astype(dtype))
    b1 = b0.copy()
    ar = None if arrays is None else [np.ascontiguousarray(a.astype(dtype)) for a in arrays]
    c = None if consts is None else np.asarray(consts, dtype=dtype)
    idx = osw.sweep(stencil, b0, b1, T, c, ar)
    return (b0, b1)[idx]


def sine_field(nx, ny, nz, h, p, q, r):
    z = np.sin(r * math.pi * np.arange(1, nz + 1) / (nz + 1))
    y = np.sin(q * math.pi * np.arange(1, ny + 1) / (ny + 1))
    x = np.sin(p * math.pi * np.arange(1, nx + 1) / (nx + 1))
    u = np.zeros((nz + 2 * h, ny + 2 * h, nx + 2 * h))
    u[h:h + nz, h:h + ny, h:h + nx] = z[:, None, None] * y[None, :, None] * x[None, None, :]
    return u


def read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split("=")
                vals[k.strip()] = float(v)
    return vals


# ---------------------------------------------------------------- eigenmodes

def lam_7c(c0, c1, nx, ny, nz, p, q, r):
    return c0 + 2 * c1 * (math.cos(p * math.pi / (nx + 1)) + math.cos(q * math.pi / (ny + 1))
                          + math.cos(r * math.pi / (nz + 1)))


def test_golden_eigenvalues_match_closed_form():
    g = read_golden("eigen_7c.txt")
    assert lam_7c(0.4, 0.1, 64, 64, 64, 1, 1, 1) == pytest.approx(g["lambda_64_p1"], abs=4e-16)
    assert lam_7c(0.4, 0.1, 64, 64, 64, 1, 1, 1) ** 16 == pytest.approx(g["lambda_64_p1_pow16"], abs=4e-15)
    assert lam_7c(0.4, 0.1, 8, 8, 8, 1, 1, 1) == pytest.approx(g["lambda_8_p1"], abs=4e-16)
    assert lam_7c(0.4, 0.1, 64, 64, 64, 64, 64, 64) == pytest.approx(g["lambda_64_p64"], abs=4e-16)


@pytest.mark.parametrize("n,T,pqr", [((64, 64, 64), 16, (1, 1, 1)), ((8, 8, 8), 16, (1, 1, 1)),
                                      ((64, 64, 64), 5, (64, 64, 64)), ((13, 7, 10), 9, (2, 3, 1)),
                                      ((10, 13, 7), 9, (5, 1, 4))])
def test_7c_sine_mode_decays_by_lambda_power(n, T, pqr):
    nx, ny, nz = n
    p, q, r = pqr
    c0, c1 = 0.4, 0.1
    u0 = sine_field(nx, ny, nz, 1, p, q, r)
    out = run("7c", u0, T, (c0, c1))
    lam = lam_7c(c0, c1, nx, ny, nz, p, q, r)
    expect = lam ** T * u0
    scale = np.max(np.abs(expect))
    assert np.max(np.abs(out - expect)) <= 1e-13 * max(scale, abs(lam) ** T * 1e-3)
    assert np.all(out[0] == 0) and np.all(out[:, 0] == 0) and np.all(out[:, :, -1] == 0)


def test_25c_sine_mode_inside_light_cone():
    nx, ny, nz, T, R = 41, 37, 43, 3, 4
    p, q, r = 2, 1, 3
    u0 = sine_field(nx, ny, nz, R, p, q, r)
    c = np.array([0.3, 0.05, 0.04, 0.03, 0.0366666])
    out = run("25c", u0, T, c)
    th = [p * math.pi / (nx + 1), q * math.pi / (ny + 1), r * math.pi / (nz + 1)]
    lam = c[0] + 2 * sum(c[m] * (math.cos(m * th[0]) + math.cos(m * th[1]) + math.cos(m * th[2]))
                         for m in range(1, 5))
    lo, reach = R, R * T
    sl = tuple(slice(lo + reach, lo + n - reach) for n in (nz, ny, nx))
    inner_out, inner_exp = out[sl], (lam ** T) * u0[sl]
    assert inner_out.size > 1000
    assert np.max(np.abs(inner_out - inner_exp)) <= 1e-13 * np.max(np.abs(inner_exp))
    # ... and outside the cone the halo has pulled the solution off the mode.
    assert np.max(np.abs(out[R:R + 2, R:-R, R:-R] - (lam ** T) * u0[R:R + 2, R:-R, R:-R])) > 1e-6


# ---------------------------------------------------------- constant field

@pytest.mark.parametrize("K", [1.0, 0.3, 0.7])
def test_7c_constant_field_preserved_bitwise(K):
    u0 = np.full((12, 11, 10), K)
    out = run("7c", u0, 16, (0.4, 0.1))
    assert np.all(out == K)


@pytest.mark.parametrize("stencil", ["7v", "25c", "25v"])
def test_normalised_constant_field_preserved(stencil):
    n = 12 if stencil.startswith("7") else 14
    h = 1 if stencil.startswith("7") else 4
    _, consts, arrays = field_and_coefs(stencil, n, n, n, seed=3)
    K, T = 0.625, 8
    u0 = np.full((n + 2 * h,) * 3, K)
    out = run(stencil, u0, T, consts, arrays)
    terms = {"7v": 13, "25c": 29, "25v": 37}[stencil]
    assert np.max(np.abs(out - K)) <= T * terms * 2.0 ** -53 * K


# ------------------------------------------------------- exact brute force

@pytest.mark.parametrize("stencil,T", [("7c", 16), ("7v", 16), ("25c", 6), ("25v", 6)])
def test_exact_rational_8cubed(stencil, T):
    u0, consts, arrays = field_and_coefs(stencil, 8, 8, 8, seed=11)
    exact = to_float(exact_sweep(stencil, u0, T, consts, arrays))
    out = run(stencil, u0, T, consts, arrays)
    terms = {"7c": 10, "7v": 13, "25c": 29, "25v": 37}[stencil]
    err = np.max(np.abs(out - exact))
    assert err <= T * terms * 2.0 ** -53 * np.max(np.abs(exact))
    assert np.linalg.norm(out - exact) <= 1e-14 * np.linalg.norm(exact)
    # the f32 oracle is the same schedule in single precision
    out32 = run(stencil, u0, T, consts, arrays, dtype=np.float32)
    assert np.max(np.abs(out32 - exact)) <= (T + 1) * terms * 2.0 ** -24 * np.max(np.abs(exact))


def test_exact_rational_nonzero_halo_and_box():
    # non-cubic box, non-zero Dirichlet halo: halo values must enter but never change
    rng = np.random.default_rng(5)
    u0 = rng.random((7 + 2, 5 + 2, 9 + 2))
    out = run("7c", u0, 7, (0.4, 0.1))
    exact = to_float(exact_sweep("7c", u0, 7, (0.4, 0.1)))
    assert np.max(np.abs(out - exact)) <= 7 * 10 * 2.0 ** -53
    h = np.ones_like(u0, dtype=bool)
    h[1:-1, 1:-1, 1:-1] = False
    assert np.array_equal(out[h], u0[h])


# ---------------------------------------------------------------- symmetry

@pytest.mark.parametrize("stencil", ["7c", "25c"])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_mirror_symmetry_bitwise(stencil, axis):
    # Listing 1 adds each +/- pair on its own, so a mirror along any axis only
    # swaps the operands of one addition: bitwise symmetric.  Listing 3 sums
    # the six radius-r neighbours in one left-to-right chain x+, x-, y+, y-,
    # z+, z-: only the x mirror (the first, commutative, addition) is bitwise;
    # y and z mirrors agree to rounding.
    n = (11, 9, 13) if stencil == "7c" else (17, 19, 18)
    u0, consts, _ = field_and_coefs(stencil, *n[::-1], seed=2)
    a = run(stencil, u0, 5, consts)
    b = run(stencil, np.ascontiguousarray(np.flip(u0, axis)), 5, consts)
    if stencil == "7c" or axis == 2:
        assert np.array_equal(np.flip(a, axis), b)
    else:
        d = np.max(np.abs(np.flip(a, axis) - b))
        assert 0 < d <= 5 * 29 * 2.0 ** -53 * np.max(np.abs(a))


# -------------------------------------------------------------- light cone

@pytest.mark.parametrize("stencil,T", [("7c", 4), ("25c", 2), ("7v", 3), ("25v", 2)])
def test_light_cone_of_impulse(stencil, T):
    R = 1 if stencil.startswith("7") else 4
    n = 2 * R * T + 5
    _, consts, arrays = field_and_coefs(stencil, n, n, n, seed=9)
    u0 = np.zeros((n + 2 * R,) * 3)
    c = R + n // 2
    u0[c, c, c] = 1.0
    out = run(stencil, u0, T, consts, arrays)
    k, j, i = np.meshgrid(*[np.arange(n + 2 * R)] * 3, indexing="ij")
    steps = sum(np.ceil(np.abs(a - c) / R) for a in (k, j, i))
    inside = steps <= T
    assert np.all(out[inside] > 0)
    assert np.all(out[~inside] == 0)


def test_impulse_near_face_never_enters_halo():
    n, T = 9, 6
    u0 = np.zeros((n + 2,) * 3)
    u0[1, 5, 5] = 1.0
    out = run("7c", u0, T, (0.4, 0.1))
    assert np.all(out[0] == 0) and out[1:-1].sum() > 0


# ---------------------------------------------------- linearity, time split

@pytest.mark.parametrize("stencil", ["7c", "7v", "25c", "25v"])
def test_linearity_and_time_split(stencil):
    n = 10 if stencil.startswith("7") else 12
    u0, consts, arrays = field_and_coefs(stencil, n, n, n, seed=4)
    v0, _, _ = field_and_coefs(stencil, n, n, n, seed=5)
    a, b = 0.75, -1.5
    lhs = run(stencil, a * u0 + b * v0, 6, consts, arrays)
    rhs = a * run(stencil, u0, 6, consts, arrays) + b * run(stencil, v0, 6, consts, arrays)
    assert np.max(np.abs(lhs - rhs)) <= 1e-14
    whole = run(stencil, u0, 7, consts, arrays)
    part = run(stencil, run(stencil, u0, 3, consts, arrays), 4, consts, arrays)
    assert np.array_equal(whole, part)


def test_result_buffer_is_T_mod_2():
    u0, consts, _ = field_and_coefs("7c", 6, 6, 6, seed=1)
    for T in (0, 1, 2, 5):
        b0, b1 = u0.copy(), u0.copy()
        idx = osw.sweep("7c", b0, b1, T, consts)
        assert idx == T % 2
        if T == 0:
            assert np.array_equal(b0, u0)


# --------------------------------------------- variable reduces to constant

def test_7v_with_constant_arrays_equals_7c():
    n = 11
    u0, _, _ = field_and_coefs("7c", n, n, n, seed=6)
    c0, c1 = 0.4, 0.1
    arrays = [np.full_like(u0, c0)] + [np.full_like(u0, c1) for _ in range(6)]
    a = run("7v", u0, 9, None, arrays)
    b = run("7c", u0, 9, (c0, c1))
    assert np.max(np.abs(a - b)) <= 1e-15 * np.max(np.abs(b)) * 9
    assert not np.array_equal(a, b) or True  # order differs; equality not required


def test_25v_with_constant_arrays_equals_25c():
    n = 13
    u0, consts, _ = field_and_coefs("25c", n, n, n, seed=7)
    arrays = [np.full_like(u0, consts[0])]
    for r in range(1, 5):
        arrays += [np.full_like(u0, consts[r])] * 3
    a = run("25v", u0, 4, None, arrays)
    b = run("25c", u0, 4, consts)
    assert np.max(np.abs(a - b)) <= 4 * 37 * 2.0 ** -53 * np.max(np.abs(b))


# ------------------------------------------------------------- arg checks

def test_oracle_rejects_bad_arguments():
    u = np.zeros((5, 5, 5))
    with pytest.raises(ValueError):
        osw.sweep("9pt", u, u.copy(), 1, (0.4, 0.1))
    with pytest.raises(ValueError):
        osw.sweep("7c", u, u.copy().astype(np.float32), 1, (0.4, 0.1))
    with pytest.raises(ValueError):
        osw.sweep("7v", u, u.copy(), 1, None, [u] * 6)


# ------------------------------------ precision: listing order, bit for bit

def numpy_listing_step(stencil, V, U, c, C, R):
    """One step of Listings 1-4 over the interior, written with whole-array
    numpy operations in the arrays' own precision (numpy keeps float32 op
    float32 in float32), in the listings' left-to-right order.  An
    independent second implementation: no loops, no C, no OpenMP."""
    nzp, nyp, nxp = V.shape
    def sh(dz, dy, dx):
        return V[R + dz:nzp - R + dz, R + dy:nyp - R + dy, R + dx:nxp - R + dx]
    inner = (slice(R, nzp - R), slice(R, nyp - R), slice(R, nxp - R))
    Vc = sh(0, 0, 0)
    if stencil == "7c":
        u = c[0] * Vc + c[1] * (sh(0, 0, 1) + sh(0, 0, -1))
        u = u + c[1] * (sh(0, 1, 0) + sh(0, -1, 0))
        u = u + c[1] * (sh(1, 0, 0) + sh(-1, 0, 0))
    elif stencil == "7v":
        Cs = [a[inner] for a in C]
        u = Cs[0] * Vc
        for m, d in enumerate([(0, 0, 1), (0, 0, -1), (0, 1, 0), (0, -1, 0), (1, 0, 0), (-1, 0, 0)]):
            u = u + Cs[m + 1] * sh(*d)
    elif stencil in ("25c", "25l"):
        b = c[0] * Vc
        for r in range(1, 5):
            s = sh(0, 0, r) + sh(0, 0, -r)
            s = s + sh(0, r, 0)
            s = s + sh(0, -r, 0)
            s = s + sh(r, 0, 0)
            s = s + sh(-r, 0, 0)
            b = b + c[r] * s
        if stencil == "25c":
            u = b
        else:
            two = V.dtype.type(2)
            u = (two * Vc - U[inner]) + C[0][inner] * b
    else:   # 25v
        Cs = [a[inner] for a in C]
        u = Cs[0] * Vc
        for r in range(1, 5):
            u = u + Cs[3 * r - 2] * (sh(0, 0, r) + sh(0, 0, -r))
            u = u + Cs[3 * r - 1] * (sh(0, r, 0) + sh(0, -r, 0))
            u = u + Cs[3 * r] * (sh(r, 0, 0) + sh(-r, 0, 0))
    assert u.dtype == V.dtype
    out = U.copy()
    out[inner] = u
    return out


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("stencil", ["7c", "7v", "25c", "25v", "25l"])
def test_oracle_equals_numpy_listing_order_bitwise(stencil, dtype):
    """The oracle's float32 (and float64) sweeps equal a whole-array numpy
    evaluation in the same precision and order, bit for bit.  A float32 sweep
    that computed in double and rounded once per point, reordered a sum or
    fused a multiply-add would differ in many elements."""
    R = 1 if stencil.startswith("7") else 4
    n = (13, 11, 9) if R == 1 else (15, 12, 11)
    u0, consts, arrays = field_and_coefs(stencil, *n, seed=21)
    u0 = u0.astype(dtype)
    c = None if consts is None else np.asarray(consts, dtype=dtype)
    C = None if arrays is None else [a.astype(dtype) for a in arrays]
    prev = u0.copy()
    if stencil == "25l":   # u^{-1} != u^0, so the U term matters
        rng = np.random.default_rng(22)
        prev[R:-R, R:-R, R:-R] = rng.random(prev[R:-R, R:-R, R:-R].shape).astype(dtype)
    T = 3
    b0, b1 = u0.copy(), prev.copy()
    idx = osw.sweep(stencil, b0, b1, T, c, C)
    got = (b0, b1)[idx]
    V, U = u0.copy(), prev.copy()
    for _ in range(T):
        U = numpy_listing_step(stencil, V, U, c, C, R)
        V, U = U, V
    assert got.dtype == dtype
    assert np.array_equal(got, V)
    if dtype == np.float32:
        # ... and differs from the float64 sweep rounded to float32 (so the
        # comparison above can tell the two precisions apart)
        b0, b1 = u0.astype(np.float64), prev.astype(np.float64)
        i64 = osw.sweep(stencil, b0, b1, T, None if c is None else c.astype(np.float64),
                        None if C is None else [a.astype(np.float64) for a in C])
        assert not np.array_equal((b0, b1)[i64].astype(np.float32), got)
