"""Pins of the oracle's 27-point box stencil (the box stencil of Section
"Handling other stencil types"; weights by distance class: c0 centre, c1 the
6 faces, c2 the 12 edges, c3 the 8 corners), each fixed by something other
than the oracle's own formula:

* a separable sine mode with zero Dirichlet halo is an eigenvector; its
  eigenvalue has the closed form
  c0 + 2 c1 (Cx+Cy+Cz) + 4 c2 (Cx Cy + Cx Cz + Cy Cz) + 8 c3 Cx Cy Cz,
  C = cos of the mode's angle per axis;
* an impulse spreads as a cube (Chebyshev distance <= t, unlike a star's
  octahedron), and the cube's corner after t steps is reached by one path
  only, all corner moves: exactly c3^t;
* dyadic weights summing to one keep a constant field bit for bit;
* with dyadic inputs every intermediate value is exact, so permuting or
  mirroring the axes of the input permutes the output exactly, the result
  equals exact rational arithmetic over the 26-neighbour box, and with the
  edge and corner weights zero it equals the pinned 7-point oracle.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import sweep as osw
from tests.exact_dyadic import exact_sweep, to_float
from workloads import field_and_coefs


def run(u0, T, c, dtype=np.float64):
    b0 = np.ascontiguousarray(u0.astype(dtype))
    b1 = b0.copy()
    idx = osw.sweep("27b", b0, b1, T, np.asarray(c, dtype=dtype))
    return (b0, b1)[idx]


def sine_field(nx, ny, nz, p, q, r):
    z = np.sin(r * math.pi * np.arange(1, nz + 1) / (nz + 1))
    y = np.sin(q * math.pi * np.arange(1, ny + 1) / (ny + 1))
    x = np.sin(p * math.pi * np.arange(1, nx + 1) / (nx + 1))
    u = np.zeros((nz + 2, ny + 2, nx + 2))
    u[1:-1, 1:-1, 1:-1] = z[:, None, None] * y[None, :, None] * x[None, None, :]
    return u


@pytest.mark.parametrize("n,T,pqr", [((12, 10, 9), 5, (1, 2, 3)), ((16, 16, 16), 8, (3, 1, 2)),
                                     ((9, 13, 11), 4, (4, 5, 2))])
def test_sine_mode_decays_by_the_closed_form_eigenvalue(n, T, pqr):
    nx, ny, nz = n
    _, c, _ = field_and_coefs("27b", 4, 4, 4, seed=3)
    cx, cy, cz = (math.cos(k * math.pi / (m + 1)) for k, m in zip(pqr, n))
    lam = c[0] + 2 * c[1] * (cx + cy + cz) + 4 * c[2] * (cx * cy + cx * cz + cy * cz) + 8 * c[3] * cx * cy * cz
    u0 = sine_field(nx, ny, nz, *pqr)
    out = run(u0, T, c)
    want = u0 * lam ** T
    assert np.max(np.abs(out - want)) <= 1e-13 * T * np.max(np.abs(u0))
    # the star operator with the same faces does not have this eigenvalue
    lam_star = c[0] + 2 * c[1] * (cx + cy + cz)
    assert abs(lam - lam_star) > 1e-3


@pytest.mark.parametrize("T", [1, 3, 5])
def test_impulse_spreads_as_a_cube_with_corner_value_c3_power_t(T):
    n = 2 * T + 5
    _, c, _ = field_and_coefs("27b", 4, 4, 4, seed=4)
    u0 = np.zeros((n + 2,) * 3)
    m = 1 + n // 2
    u0[m, m, m] = 1.0
    out = run(u0, T, c)
    k, j, i = np.meshgrid(*[np.arange(n + 2)] * 3, indexing="ij")
    cheb = np.maximum(np.maximum(np.abs(k - m), np.abs(j - m)), np.abs(i - m))
    assert np.all(out[cheb <= T] > 0)
    assert np.all(out[cheb > T] == 0)
    corner = 1.0
    for _ in range(T):
        corner = corner * c[3]
    for sk, sj, si in itertools.product((-1, 1), repeat=3):
        assert out[m + sk * T, m + sj * T, m + si * T] == corner


def test_constant_field_preserved_bitwise():
    c = [1 / 8, 1 / 16, 1 / 64, 5 / 128]
    assert c[0] + 6 * c[1] + 12 * c[2] + 8 * c[3] == 1.0
    u0 = np.full((11, 10, 12), 3.0)
    for dtype in (np.float64, np.float32):
        assert np.array_equal(run(u0, 6, c, dtype), u0.astype(dtype))


def dyadic_input(n, seed):
    rng = np.random.default_rng(seed)
    u0 = np.zeros((n[2] + 2, n[1] + 2, n[0] + 2))
    u0[1:-1, 1:-1, 1:-1] = rng.integers(-64, 64, size=(n[2], n[1], n[0])) / 64.0
    return u0


DYADIC_C = [1 / 4, 3 / 32, -1 / 64, 1 / 128]


@pytest.mark.parametrize("perm", [(0, 2, 1), (1, 0, 2), (2, 1, 0), (1, 2, 0)])
def test_axis_permutations_and_mirrors_commute_exactly(perm):
    u0 = dyadic_input((9, 8, 7), 5)
    a = run(u0, 3, DYADIC_C)
    b = run(np.ascontiguousarray(np.transpose(u0, perm)), 3, DYADIC_C)
    assert np.array_equal(np.transpose(a, perm), b)
    for axis in range(3):
        m = run(np.ascontiguousarray(np.flip(u0, axis)), 3, DYADIC_C)
        assert np.array_equal(np.flip(a, axis), m)


def test_equals_exact_rational_box():
    u0 = dyadic_input((7, 6, 5), 6)
    exact = to_float(exact_sweep("27b", u0, 3, DYADIC_C))
    assert np.array_equal(run(u0, 3, DYADIC_C), exact)
    # random (non-dyadic) inputs: within the rounding of 30 operations a step
    u0, c, _ = field_and_coefs("27b", 8, 7, 6, seed=7)
    exact = to_float(exact_sweep("27b", u0, 4, c))
    out = run(u0, 4, c)
    assert np.max(np.abs(out - exact)) <= 4 * 30 * 2.0 ** -53 * np.max(np.abs(exact))
    out32 = run(u0, 4, c, np.float32)
    assert np.max(np.abs(out32 - exact)) <= 5 * 30 * 2.0 ** -24 * np.max(np.abs(exact))


def test_faces_only_equal_the_seven_point_stencil():
    u0 = dyadic_input((8, 9, 7), 8)
    box = run(u0, 3, [1 / 4, 1 / 8, 0.0, 0.0])
    b0 = u0.copy()
    b1 = u0.copy()
    idx = osw.sweep("7c", b0, b1, 3, np.array([1 / 4, 1 / 8]))
    assert np.array_equal(box, (b0, b1)[idx])


def test_planted_misclassification_is_caught():
    """An oracle that weighted the edges as corners would fail the eigenmode
    pin: its eigenvalue differs from the closed form."""
    _, c, _ = field_and_coefs("27b", 4, 4, 4, seed=3)
    cx, cy, cz = (math.cos(k * math.pi / (m + 1)) for k, m in zip((1, 2, 3), (12, 10, 9)))
    good = c[0] + 2 * c[1] * (cx + cy + cz) + 4 * c[2] * (cx * cy + cx * cz + cy * cz) + 8 * c[3] * cx * cy * cz
    swapped = c[0] + 2 * c[1] * (cx + cy + cz) + 4 * c[3] * (cx * cy + cx * cz + cy * cz) + 8 * c[2] * cx * cy * cz
    assert abs(good - swapped) > 1e-3
