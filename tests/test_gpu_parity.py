"""GPU parity: the HIP naive sweep and the HIP diamond/wavefront (MWD) sweep
against the CPU oracle, element by element, through the C ABI.

Bar (from the method: blocking only reorders point updates, every kernel
evaluates the listings' order without contraction):
  * naive GPU == oracle, bit for bit (float64 and float32 oracles);
  * MWD GPU == naive GPU == oracle, bit for bit;
  * float64 MWD within 1e-12 relative L2 of the float64 oracle (implied).
Sizes span several x-chunks, several diamonds and rows, ragged tails in every
axis, T below, at and above the diamond height, and the degenerate cases
(T = 0, T = 1, grids thinner than a diamond).  The second buffer's interior is
poisoned with NaN: a schedule that reads a value it did not produce fails.
"""
import numpy as np
import pytest

from tests.gpu_util import inputs, oracle_run, run_gpu

pytestmark = pytest.mark.gpu


def assert_bitwise(a, b, what):
    if not np.array_equal(a, b):
        bad = np.argwhere(~((a == b) | (np.isnan(a) & np.isnan(b))))
        raise AssertionError("%s: %d elements differ, first at %s: %r vs %r"
                             % (what, len(bad), bad[:3].tolist(), a[tuple(bad[0])], b[tuple(bad[0])]))


CASES_NAIVE = [("7c", (37, 29, 23), 5), ("7v", (35, 19, 21), 4), ("25c", (45, 37, 29), 3), ("25v", (41, 35, 33), 2),
               ("25l", (43, 37, 31), 3), ("27b", (37, 29, 23), 5), ("27b", (130, 7, 66), 3), ("27b", (1, 1, 1), 2)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("stencil,n,T", CASES_NAIVE)
def test_naive_matches_oracle_bitwise(stencil, n, T, dtype):
    u0, c, arr = inputs(stencil, *n, seed=1)
    print("naive", stencil, dtype, n, T, flush=True)
    got, _ = run_gpu(stencil, dtype, u0, c, arr, T, algo="naive")
    ref = oracle_run(stencil, u0, c, arr, T, dtype)
    assert_bitwise(got, ref, "naive %s %s" % (stencil, dtype))


def test_naive_block_shapes():
    u0, c, arr = inputs("7c", 70, 33, 41, seed=2)
    ref = oracle_run("7c", u0, c, arr, 3)
    for p in ({"threads_x": 128, "threads_y": 2, "tile_z": 7}, {"threads_x": 64, "threads_y": 1, "tile_z": 200},
              {"threads_x": 256, "threads_y": 1, "tile_z": 16}):
        got, _ = run_gpu("7c", "f64", u0, c, arr, 3, algo="naive", params=p)
        assert_bitwise(got, ref, "naive %s" % p)


def test_box_block_shapes_halo_and_pitch():
    """The 27-point box stencil's naive sweep: several block shapes and z
    chunks, a nonzero halo with a -0.0 (diagonal neighbours reach the halo's
    edges and corners), and padded pitches, bit for bit against the oracle."""
    u0, c, arr = inputs("27b", 70, 33, 41, seed=2)
    rng = np.random.default_rng(2)
    halo = np.ones(u0.shape, bool)
    halo[1:-1, 1:-1, 1:-1] = False
    u0[halo] = rng.random(int(halo.sum())) - 0.5
    u0[0, 0, 0] = -0.0
    for dtype in ("f64", "f32"):
        ref = oracle_run("27b", u0, c, arr, 4, dtype)
        for p in ({"threads_x": 128, "threads_y": 2, "tile_z": 7}, {"threads_x": 64, "threads_y": 1, "tile_z": 200},
                  {"threads_x": 256, "threads_y": 1, "tile_z": 16}, None):
            print("box", dtype, p, flush=True)
            got, _ = run_gpu("27b", dtype, u0, c, arr, 4, algo="naive", params=p)
            assert_bitwise(got, ref, "box %s %s" % (dtype, p))
        got, _ = run_gpu("27b", dtype, u0, c, arr, 4, algo="naive", pitch=(80, 40))
        assert_bitwise(got, ref, "box padded %s" % dtype)


def test_box_register_columns():
    """The box stencil's register-column sweep (variant 1) in every compiled
    shape (2 or 4 waves, 2, 4 or 8 rows per lane), with z chunks that do and
    do not divide nz, a nonzero halo with a -0.0, padded pitches, and grids
    whose x extent falls on, just below and just above the 62 cells a wave
    stores, bit for bit against the oracle."""
    u0, c, arr = inputs("27b", 70, 33, 41, seed=4)
    rng = np.random.default_rng(4)
    halo = np.ones(u0.shape, bool)
    halo[1:-1, 1:-1, 1:-1] = False
    u0[halo] = rng.random(int(halo.sum())) - 0.5
    u0[0, 0, 0] = -0.0
    for dtype in ("f64", "f32"):
        ref = oracle_run("27b", u0, c, arr, 4, dtype)
        for w in (2, 4):
            for ky in (2, 4, 8):
                for tz in (7, 41, 200):
                    p = {"variant": 1, "threads_x": 64, "threads_y": w, "cells_per_lane": ky, "tile_z": tz}
                    print("box columns", dtype, p, flush=True)
                    got, info = run_gpu("27b", dtype, u0, c, arr, 4, algo="naive", params=p)
                    assert (info["params"]["tile_y"], info["params"]["cells_per_lane"]) == (w * ky, ky)
                    assert_bitwise(got, ref, "box columns %s %s" % (dtype, p))
        got, _ = run_gpu("27b", dtype, u0, c, arr, 4, algo="naive", pitch=(80, 40))
        assert_bitwise(got, ref, "box columns padded %s" % dtype)
    for n in ((61, 5, 9), (62, 16, 3), (63, 17, 4), (1, 1, 1), (130, 47, 12), (124, 1, 2), (2, 70, 5)):
        u0, c, arr = inputs("27b", *n, seed=5)
        for dtype in ("f64", "f32"):
            print("box columns grid", dtype, n, flush=True)
            got, _ = run_gpu("27b", dtype, u0, c, arr, 5, algo="naive")
            assert_bitwise(got, oracle_run("27b", u0, c, arr, 5, dtype), "box columns %s %s" % (dtype, n))


@pytest.mark.parametrize("stencil", ["7c", "25c"])
def test_star_register_columns(stencil):
    """Naive variant 2 (register columns) of the constant-coefficient star
    stencils in every compiled shape (2 or 4 waves, 2, 4 or 8 rows per lane),
    z chunks that do and do not divide nz, a nonzero halo with a -0.0,
    padded pitches, and grids whose extents fall on, below and above the
    64 - 2R x cells and the rows a wave stores, bit for bit against the
    oracle."""
    h = 1 if stencil == "7c" else 4
    u0, c, arr = inputs(stencil, 70, 33, 41, seed=6)
    rng = np.random.default_rng(6)
    halo = np.ones(u0.shape, bool)
    halo[h:-h, h:-h, h:-h] = False
    u0[halo] = rng.random(int(halo.sum())) - 0.5
    u0[0, 0, 0] = -0.0
    for dtype in ("f64", "f32"):
        ref = oracle_run(stencil, u0, c, arr, 4, dtype)
        for w in (2, 4):
            for ky in (2, 4, 8):
                for tz in (5, 41):
                    p = {"variant": 2, "threads_x": 64, "threads_y": w, "cells_per_lane": ky, "tile_z": tz}
                    print("star columns", stencil, dtype, p, flush=True)
                    got, info = run_gpu(stencil, dtype, u0, c, arr, 4, algo="naive", params=p)
                    assert (info["params"]["variant"], info["params"]["tile_x"]) == (2, 64 - 2 * h)
                    assert_bitwise(got, ref, "star columns %s %s %s" % (stencil, dtype, p))
        p = {"variant": 2, "threads_x": 64, "threads_y": 4, "cells_per_lane": 4}
        got, _ = run_gpu(stencil, dtype, u0, c, arr, 4, algo="naive", params=p, pitch=(80 + 2 * h, 40 + 2 * h))
        assert_bitwise(got, ref, "star columns padded %s %s" % (stencil, dtype))
    own = 64 - 2 * h
    for n in ((own - 1, 9, 7), (own, 16, 3), (own + 1, 17, 4), (1, 1, 1), (130, 47, 12), (2, 70, 9), (3, 5, 1)):
        u0, c, arr = inputs(stencil, *n, seed=7)
        for dtype in ("f64", "f32"):
            for ky in (2, 8):
                p = {"variant": 2, "threads_x": 64, "threads_y": 2, "cells_per_lane": ky}
                print("star columns grid", stencil, dtype, n, p, flush=True)
                got, _ = run_gpu(stencil, dtype, u0, c, arr, 5, algo="naive", params=p)
                assert_bitwise(got, oracle_run(stencil, u0, c, arr, 5, dtype),
                               "star columns %s %s %s %s" % (stencil, dtype, n, p))


@pytest.mark.parametrize("stencil", ["7c", "7v", "25c", "25v", "25l"])
def test_naive_plane_tiles_bitwise(stencil):
    """The LDS-tile naive sweep (variant 1) at every compiled tile height, on
    grids whose x and y are not multiples of the tile and z chunks that do not
    divide nz, equals the oracle in FP64 and FP32."""
    n = (70, 37, 23) if stencil.startswith("7") else (135, 41, 19)
    u0, c, arr = inputs(stencil, *n, seed=5)
    for dtype in ("f64", "f32"):
        ref = oracle_run(stencil, u0, c, arr, 3, dtype)
        for rows, tz in ((4, 7), (8, 64), (16, 5)):
            p = {"variant": 1, "threads_x": 64, "threads_y": rows, "tile_z": tz}
            print("naive tiles", stencil, dtype, p, flush=True)
            got, info = run_gpu(stencil, dtype, u0, c, arr, 3, algo="naive", params=p)
            assert info["params"]["variant"] == 1
            assert_bitwise(got, ref, "naive tiles %s %s %s" % (stencil, dtype, p))


def test_leapfrog_with_initial_velocity_bitwise():
    """The second-order-in-time stencil reads buf1 as u^{-1}: with u^{-1} != u^0
    both naive variants follow the oracle bit for bit, in FP64 and FP32."""
    n = (69, 33, 27)
    u0, c, arr = inputs("25l", *n, seed=7)
    rng = np.random.default_rng(8)
    prev = u0.copy()
    prev[4:-4, 4:-4, 4:-4] = rng.random(n[::-1])
    for dtype in ("f64", "f32"):
        ref = oracle_run("25l", u0, c, arr, 5, dtype, prev=prev)
        for p in ({"variant": 0, "threads_x": 64, "threads_y": 4, "tile_z": 9},
                  {"variant": 1, "threads_x": 64, "threads_y": 8, "tile_z": 16}):
            got, _ = run_gpu("25l", dtype, u0, c, arr, 5, algo="naive", params=p, prev=prev)
            assert_bitwise(got, ref, "leapfrog %s %s" % (dtype, p))


def leapfrog_prev(u0, seed):
    """u^{-1}: u^0's halo, a random interior."""
    rng = np.random.default_rng(seed)
    prev = u0.copy()
    prev[4:-4, 4:-4, 4:-4] = rng.random(tuple(d - 8 for d in u0.shape))
    return prev


# Second-order-in-time 25-point stencil, blocked (dtype, Dw, cells per lane,
# waves along x, N_F, tile_x or 0, grid, list of T): every compiled shape,
# u^{-1} != u^0, T from one step to several rows, with even and odd numbers
# of diamond rows (an odd count starts from the plan's own pair, which then
# receives both input levels)
MWD_LEAPFROG_CASES = [
    ("f64", 16, 1, 1, 1, 0, (150, 50, 22), [1, 2, 3, 5, 11]),
    ("f64", 16, 1, 1, 1, 40, (131, 37, 19), [4, 7]),
    ("f64", 8, 1, 2, 1, 0, (140, 30, 20), [1, 2, 3, 6]),
    ("f32", 16, 1, 1, 1, 0, (100, 45, 21), [2, 3, 7]),
    ("f32", 16, 1, 1, 2, 0, (100, 45, 21), [1, 4, 9]),
    ("f32", 16, 1, 1, 2, 0, (70, 20, 8), [3, 6]),
    ("f32", 8, 1, 2, 1, 0, (140, 30, 20), [3, 5]),
]


@pytest.mark.parametrize("dtype,dw,vx,wx,nf,tx,n,Ts", MWD_LEAPFROG_CASES)
def test_mwd_leapfrog_bitwise(dtype, dw, vx, wx, nf, tx, n, Ts):
    u0, c, arr = inputs("25l", *n, seed=9)
    prev = leapfrog_prev(u0, 10)
    params = mwd_params(dw, vx, wx, tx, nf)
    for T in Ts:
        print("mwd leapfrog", dtype, dw, vx, wx, nf, tx, n, T, flush=True)
        got, info = run_gpu("25l", dtype, u0, c, arr, T, algo="mwd", params=params, prev=prev)
        q = info["params"]
        assert (q["diamond_width"], q["wavefront_depth"]) == (dw, nf)
        assert_bitwise(got, oracle_run("25l", u0, c, arr, T, dtype, prev=prev),
                       "mwd leapfrog %s Dw=%d nf=%d T=%d" % (dtype, dw, nf, T))
        naive, _ = run_gpu("25l", dtype, u0, c, arr, T, algo="naive", prev=prev)
        assert_bitwise(got, naive, "mwd leapfrog vs naive")


def test_mwd_leapfrog_schedules_halo_and_thin_grids():
    """The blocked second-order stencil with the dependency-driven schedule,
    a nonzero halo (the general-halo instance), and grids thinner than a
    diamond or a slab."""
    params = mwd_params(16, 1, 1)
    u0, c, arr = inputs("25l", 120, 44, 23, seed=11)
    prev = leapfrog_prev(u0, 12)
    for T in (1, 4, 9):
        print("mwd leapfrog sweep", T, flush=True)
        got, _ = run_gpu("25l", "f64", u0, c, arr, T, algo="mwd", params=dict(params, variant=1), prev=prev,
                         check=True)
        assert_bitwise(got, oracle_run("25l", u0, c, arr, T, "f64", prev=prev), "leapfrog sweep T=%d" % T)
    u0, c, arr = inputs("25l", 60, 30, 14, seed=13)
    rng = np.random.default_rng(13)
    halo = np.ones(u0.shape, bool)
    halo[4:-4, 4:-4, 4:-4] = False
    u0[halo] = rng.random(int(halo.sum())) - 0.5
    prev = leapfrog_prev(u0, 14)
    for dtype, nf in (("f64", 1), ("f32", 2)):
        print("mwd leapfrog nonzero halo", dtype, flush=True)
        got, _ = run_gpu("25l", dtype, u0, c, arr, 5, algo="mwd", params=mwd_params(16, 1, 1, 0, nf), prev=prev)
        assert_bitwise(got, oracle_run("25l", u0, c, arr, 5, dtype, prev=prev), "leapfrog nonzero halo %s" % dtype)
    for n in ((9, 5, 3), (1, 1, 1), (33, 7, 2)):
        u0, c, arr = inputs("25l", *n, seed=15)
        prev = leapfrog_prev(u0, 16)
        print("mwd leapfrog thin", n, flush=True)
        got, _ = run_gpu("25l", "f64", u0, c, arr, 6, algo="mwd", prev=prev)
        assert_bitwise(got, oracle_run("25l", u0, c, arr, 6, "f64", prev=prev), "leapfrog thin %s" % (n,))


# (stencil, dtype, Dw, cells per lane, waves along x, tile_x or 0, grid (nx, ny, nz), list of T):
# every compiled MWD variant at least once, each grid several x chunks wide
MWD_CASES = [
    ("7c", "f64", 4, 2, 2, 0, (300, 23, 17), [1, 2, 3, 5, 8]),
    ("7c", "f64", 8, 1, 2, 0, (150, 45, 19), [1, 4, 5, 9, 13]),
    ("7c", "f64", 8, 1, 3, 0, (400, 45, 19), [5, 9]),
    ("7c", "f32", 8, 1, 3, 100, (400, 33, 15), [4]),
    ("7c", "f32", 8, 1, 4, 40, (150, 45, 19), [7]),
    ("7c", "f64", 8, 2, 1, 0, (150, 45, 19), [4, 9]),
    ("7c", "f64", 8, 2, 2, 0, (300, 33, 15), [5, 12]),
    ("7c", "f64", 12, 1, 2, 0, (131, 50, 12), [6, 7, 16]),
    ("7c", "f64", 12, 1, 2, 40, (131, 50, 12), [7]),
    ("7c", "f32", 12, 2, 1, 0, (200, 40, 11), [9, 16]),
    ("7c", "f64", 16, 1, 1, 0, (70, 70, 9), [3, 8, 17]),
    ("7c", "f32", 16, 1, 1, 0, (200, 40, 11), [9, 16]),
    ("7c", "f32", 16, 2, 1, 0, (260, 37, 9), [10]),
    ("7c", "f32", 4, 2, 2, 0, (300, 23, 17), [3]),
    ("7v", "f64", 8, 1, 2, 0, (129, 30, 14), [3, 7]),
    ("7v", "f64", 8, 1, 3, 0, (200, 41, 10), [6, 11]),
    ("7v", "f64", 8, 2, 1, 0, (260, 33, 12), [5, 9]),
    ("7v", "f32", 8, 1, 2, 0, (129, 30, 14), [4]),
    ("7v", "f32", 8, 1, 4, 30, (150, 25, 11), [5]),
    ("7v", "f32", 8, 2, 1, 0, (260, 33, 12), [9]),
    ("7v", "f32", 12, 1, 2, 0, (120, 41, 10), [6, 11]),
    ("7v", "f32", 12, 2, 1, 0, (200, 30, 9), [7]),
    ("7v", "f32", 16, 1, 1, 0, (120, 41, 10), [9]),
    ("25c", "f64", 8, 1, 2, 0, (140, 30, 20), [1, 2, 3]),
    ("25c", "f32", 8, 1, 4, 0, (300, 30, 20), [2, 5]),
    ("25c", "f64", 8, 2, 1, 0, (140, 30, 20), [3]),
    ("25c", "f64", 16, 1, 1, 0, (150, 50, 22), [2, 3, 5]),
    ("25c", "f32", 16, 2, 1, 0, (260, 45, 17), [4]),
    ("25c", "f32", 24, 1, 1, 0, (100, 60, 21), [3, 7]),
    ("25c", "f32", 8, 2, 2, 0, (600, 30, 20), [2, 5]),
    ("25v", "f64", 8, 1, 2, 0, (130, 40, 19), [2, 5]),
    ("25v", "f64", 8, 1, 1, 0, (70, 33, 17), [3]),
    ("25v", "f64", 8, 2, 1, 0, (250, 26, 18), [1, 4]),
    ("25v", "f32", 8, 1, 2, 0, (130, 40, 19), [3]),
    ("25v", "f32", 8, 2, 1, 0, (250, 26, 18), [3]),
    ("25v", "f32", 16, 1, 1, 0, (100, 45, 21), [2, 3, 7]),
    ("27b", "f64", 8, 1, 2, 0, (150, 45, 19), [1, 2, 3, 4, 5, 9, 13]),
    ("27b", "f64", 8, 1, 2, 22, (131, 37, 21), [6]),
    ("27b", "f32", 8, 1, 2, 0, (140, 30, 20), [3, 8]),
    ("27b", "f32", 12, 1, 2, 0, (200, 50, 25), [1, 5, 7, 14]),
    ("27b", "f32", 12, 1, 2, 40, (131, 50, 12), [7, 16]),
]


def mwd_params(dw, vx, wx, tx=0, nf=1):
    return {"diamond_width": dw, "cells_per_lane": vx, "threads_x": 64 * wx, "tile_x": tx, "wavefront_depth": nf}


@pytest.mark.parametrize("stencil,dtype,dw,vx,wx,tx,n,Ts", MWD_CASES)
def test_mwd_matches_naive_and_oracle_bitwise(stencil, dtype, dw, vx, wx, tx, n, Ts):
    u0, c, arr = inputs(stencil, *n, seed=3)
    params = mwd_params(dw, vx, wx, tx)
    for T in Ts:
        print("mwd", stencil, dtype, dw, vx, wx, tx, n, T, flush=True)
        got, info = run_gpu(stencil, dtype, u0, c, arr, T, algo="mwd", params=params)
        q = info["params"]
        assert (q["diamond_width"], q["cells_per_lane"], q["threads_x"]) == (dw, vx, 64 * wx)
        ref = oracle_run(stencil, u0, c, arr, T, dtype)
        assert_bitwise(got, ref, "mwd %s %s Dw=%d vx=%d wx=%d T=%d" % (stencil, dtype, dw, vx, wx, T))
        naive, _ = run_gpu(stencil, dtype, u0, c, arr, T, algo="naive")
        assert_bitwise(got, naive, "mwd vs naive")
        if dtype == "f64":
            assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


# Wavefront depth N_F > 1 (NF planes per wavefront step): every compiled
# variant on grids whose nz is odd and even, several x chunks, T below, at and
# above the diamond height (stencil, dtype, Dw, cells per lane, waves along x,
# N_F, tile_x or 0, grid, list of T)
MWD_NF_CASES = [
    ("7c", "f64", 8, 1, 2, 2, 0, (150, 45, 19), [1, 4, 5, 9, 13]),
    ("7c", "f64", 8, 1, 2, 2, 0, (131, 50, 12), [7, 16]),
    ("7c", "f32", 12, 1, 2, 2, 0, (131, 50, 13), [6, 7, 16]),
    ("7c", "f32", 12, 1, 2, 2, 40, (131, 37, 8), [11]),
    ("7c", "f32", 16, 1, 1, 2, 0, (70, 70, 9), [3, 8, 17]),
    ("7c", "f32", 8, 1, 2, 2, 0, (150, 45, 20), [5, 9]),
    ("25c", "f32", 16, 1, 1, 2, 0, (100, 45, 21), [1, 4, 7]),
    ("25c", "f32", 16, 1, 1, 2, 0, (100, 45, 24), [2, 5]),
    ("7v", "f64", 8, 1, 2, 2, 0, (129, 30, 15), [3, 7]),
    ("7v", "f32", 8, 1, 2, 2, 0, (129, 30, 14), [4, 9]),
]


@pytest.mark.parametrize("stencil,dtype,dw,vx,wx,nf,tx,n,Ts", MWD_NF_CASES)
def test_mwd_wavefront_depth_matches_naive_and_oracle_bitwise(stencil, dtype, dw, vx, wx, nf, tx, n, Ts):
    u0, c, arr = inputs(stencil, *n, seed=13)
    params = mwd_params(dw, vx, wx, tx, nf)
    for T in Ts:
        print("mwd nf", stencil, dtype, dw, vx, wx, nf, tx, n, T, flush=True)
        got, info = run_gpu(stencil, dtype, u0, c, arr, T, algo="mwd", params=params)
        q = info["params"]
        assert (q["diamond_width"], q["cells_per_lane"], q["threads_x"], q["wavefront_depth"]) == (dw, vx, 64 * wx, nf)
        ref = oracle_run(stencil, u0, c, arr, T, dtype)
        assert_bitwise(got, ref, "mwd %s %s Dw=%d vx=%d wx=%d nf=%d T=%d" % (stencil, dtype, dw, vx, wx, nf, T))


@pytest.mark.parametrize("stencil,dtype,dw,vx,wx,nf", [("7c", "f64", 8, 1, 2, 2), ("7c", "f32", 12, 1, 2, 2),
                                                      ("25c", "f32", 16, 1, 1, 2)])
def test_mwd_wavefront_depth_thin_and_nonzero_halo(stencil, dtype, dw, vx, wx, nf):
    """Grids thinner than a slab or a diamond (nz = 1, 2, 3), and a nonzero
    Dirichlet halo (with a -0.0), at N_F > 1."""
    for n in ((9, 5, 1), (70, 3, 2), (33, 17, 3)):
        u0, c, arr = inputs(stencil, *n, seed=14)
        for T in (1, 5):
            got, _ = run_gpu(stencil, dtype, u0, c, arr, T, algo="mwd", params=mwd_params(dw, vx, wx, 0, nf))
            assert_bitwise(got, oracle_run(stencil, u0, c, arr, T, dtype), "thin %s nf=%d %s T=%d" % (stencil, nf, n, T))
    u0, c, arr = inputs(stencil, 131, 29, 11, seed=8)
    h = 1 if stencil.startswith("7") else 4
    rng = np.random.default_rng(3)
    halo = np.ones(u0.shape, dtype=bool)
    halo[h:-h, h:-h, h:-h] = False
    u0 = u0.copy()
    u0[halo] = rng.random(int(halo.sum())) - 0.5
    u0[0, 0, 0] = -0.0
    got, _ = run_gpu(stencil, dtype, u0, c, arr, 7, algo="mwd", params=mwd_params(dw, vx, wx, 0, nf))
    assert_bitwise(got, oracle_run(stencil, u0, c, arr, 7, dtype), "nonzero halo %s nf=%d" % (stencil, nf))


# Dependency-driven schedule (variant 1: one launch, each tile starts when
# the tiles of the previous row it depends on are done): every shape compiled
# with it, on grids with one and several x chunks and diamonds, T from one
# row to many (stencil, dtype, Dw, cells per lane, waves along x, N_F,
# tile_x or 0, grid, list of T)
MWD_SWEEP_CASES = [
    ("7c", "f64", 12, 1, 2, 1, 0, (300, 70, 17), [1, 5, 6, 7, 13, 40]),
    ("7c", "f64", 12, 1, 2, 1, 40, (131, 50, 12), [9, 16]),
    ("7c", "f64", 8, 1, 2, 1, 0, (150, 45, 19), [4, 9, 21]),
    ("7c", "f32", 12, 1, 2, 1, 0, (200, 40, 11), [9, 16]),
    ("7c", "f32", 12, 1, 2, 2, 0, (131, 50, 13), [6, 7, 30]),
    ("25c", "f64", 16, 1, 1, 1, 0, (150, 50, 22), [2, 3, 5, 11]),
    ("25c", "f32", 16, 2, 1, 1, 0, (260, 45, 17), [4, 9]),
    ("25c", "f32", 16, 1, 1, 2, 0, (100, 45, 21), [1, 4, 7]),
    ("7v", "f64", 8, 1, 2, 1, 0, (129, 30, 14), [3, 7, 12]),
    ("7v", "f32", 12, 1, 2, 1, 0, (120, 41, 10), [6, 11]),
]


@pytest.mark.parametrize("stencil,dtype,dw,vx,wx,nf,tx,n,Ts", MWD_SWEEP_CASES)
def test_mwd_dependency_driven_schedule_bitwise(stencil, dtype, dw, vx, wx, nf, tx, n, Ts):
    u0, c, arr = inputs(stencil, *n, seed=17)
    params = dict(mwd_params(dw, vx, wx, tx, nf), variant=1)
    for T in Ts:
        print("mwd sweep", stencil, dtype, dw, vx, wx, nf, tx, n, T, flush=True)
        got, info = run_gpu(stencil, dtype, u0, c, arr, T, algo="mwd", params=params, check=True)
        assert info["params"]["variant"] == 1
        assert_bitwise(got, oracle_run(stencil, u0, c, arr, T, dtype),
                       "sweep %s %s Dw=%d vx=%d wx=%d nf=%d T=%d" % (stencil, dtype, dw, vx, wx, nf, T))


# Relaxed synchronisation within the tile (variant bit 1: per-wave step
# counters instead of barriers), with row launches (2) and with the
# dependency-driven schedule (3), for every shape compiled with it; the
# non-zero halo case runs the general-halo instance, which keeps the barriers.
MWD_RELAX_CASES = [
    ("7c", "f64", 12, 1, 2, 1, 0, (300, 70, 17), [1, 5, 6, 7, 13, 40]),
    ("7c", "f64", 12, 1, 2, 1, 40, (131, 50, 12), [9, 16]),
    ("7c", "f64", 12, 1, 2, 1, 0, (70, 13, 5), [3, 12]),
    ("7c", "f32", 12, 1, 2, 2, 0, (131, 50, 13), [6, 7, 30]),
    ("7c", "f32", 12, 1, 2, 2, 0, (260, 37, 9), [1, 11]),
]


@pytest.mark.parametrize("variant", [2, 3])
@pytest.mark.parametrize("stencil,dtype,dw,vx,wx,nf,tx,n,Ts", MWD_RELAX_CASES)
def test_mwd_relaxed_synchronisation_bitwise(stencil, dtype, dw, vx, wx, nf, tx, n, Ts, variant):
    u0, c, arr = inputs(stencil, *n, seed=19)
    params = dict(mwd_params(dw, vx, wx, tx, nf), variant=variant)
    for T in Ts:
        print("mwd relaxed", variant, stencil, dtype, dw, vx, wx, nf, tx, n, T, flush=True)
        got, info = run_gpu(stencil, dtype, u0, c, arr, T, algo="mwd", params=params, check=True)
        assert info["params"]["variant"] == variant
        assert_bitwise(got, oracle_run(stencil, u0, c, arr, T, dtype),
                       "relaxed v%d %s %s Dw=%d nf=%d T=%d" % (variant, stencil, dtype, dw, nf, T))


@pytest.mark.parametrize("dtype,nf", [("f64", 1), ("f32", 2)])
def test_mwd_relaxed_synchronisation_nonzero_halo(dtype, nf):
    n = (90, 40, 15)
    u0, c, arr = inputs("7c", *n, seed=20)
    rng = np.random.default_rng(20)
    halo = np.ones(u0.shape, bool)
    halo[1:-1, 1:-1, 1:-1] = False
    u0[halo] = rng.random(int(halo.sum())) - 0.5
    params = dict(mwd_params(12, 1, 2, 0, nf), variant=2)
    print("mwd relaxed nonzero halo", dtype, nf, flush=True)
    got, _ = run_gpu("7c", dtype, u0, c, arr, 9, algo="mwd", params=params, check=True)
    assert_bitwise(got, oracle_run("7c", u0, c, arr, 9, dtype), "relaxed nonzero halo %s" % dtype)


def test_relaxed_waits_that_give_up_are_reported():
    """A wait limit of zero polls makes a wave give up at its first wait that
    finds a neighbour behind (among the many waits of a 30-step run some
    do): the launch ends, girih_check reports GIRIH_E_STALL, and with the
    default limit the plan then computes the oracle's result."""
    import paper_1510_04995_amd as P
    import paper_1510_04995_amd.girih as G
    from tests.gpu_util import torch_dev, upload
    torch, dev = torch_dev()
    n = (150, 60, 40)
    u0, c, arr = inputs("7c", *n, seed=21)
    sw = P.Sweep("7c", "f64", *n, list(c), "mwd", {"variant": 2})
    sw.set_wait_limit(0)
    b0, b1 = upload(u0), upload(u0)
    print("relaxed stall", flush=True)
    sw.run(b0, b1, 30)
    with pytest.raises(G.GirihError) as e:
        sw.check()
    assert e.value.code == G.E_STALL
    sw.set_wait_limit(1 << 20)
    b0, b1 = upload(u0), upload(u0)
    out = sw.run(b0, b1, 30)
    sw.check()
    assert_bitwise(out.cpu().numpy(), oracle_run("7c", u0, c, arr, 30), "after a stalled relaxed run")
    sw.close()


def test_dependency_waits_that_give_up_are_reported():
    """With a wait limit of zero polls, tiles of the second and later rows give
    up at once (every tile of this small grid is resident together), the
    launch still ends and girih_check reports GIRIH_E_STALL; with the default
    limit the same plan then computes the oracle's result."""
    import paper_1510_04995_amd as P
    import paper_1510_04995_amd.girih as G
    from tests.gpu_util import torch_dev, upload
    torch, dev = torch_dev()
    n = (150, 60, 40)
    u0, c, arr = inputs("7c", *n, seed=18)
    sw = P.Sweep("7c", "f64", *n, list(c), "mwd", {"diamond_width": 12, "threads_x": 128, "variant": 1})
    sw.set_wait_limit(0)
    b0, b1 = upload(u0), upload(u0)
    sw.run(b0, b1, 30)
    with pytest.raises(G.GirihError) as e:
        sw.check()
    assert e.value.code == G.E_STALL
    sw.set_wait_limit(1 << 20)
    b0, b1 = upload(u0), upload(u0)
    out = sw.run(b0, b1, 30)
    sw.check()
    assert_bitwise(out.cpu().numpy(), oracle_run("7c", u0, c, arr, 30), "after a stalled run")
    sw.close()


def test_mwd_T0_and_T1_and_tiny_grids():
    for n in ((1, 1, 1), (3, 2, 5), (9, 1, 4), (2, 17, 1)):
        u0, c, arr = inputs("7c", *n, seed=4)
        for T in (0, 1, 2, 9):
            got, _ = run_gpu("7c", "f64", u0, c, arr, T, algo="mwd", params={"diamond_width": 8})
            assert_bitwise(got, oracle_run("7c", u0, c, arr, T), "tiny %s T=%d" % (n, T))
    u0, c, arr = inputs("25c", 5, 3, 6, seed=4)
    got, _ = run_gpu("25c", "f64", u0, c, arr, 3, algo="mwd", params={"diamond_width": 16})
    assert_bitwise(got, oracle_run("25c", u0, c, arr, 3), "tiny 25c")


@pytest.mark.parametrize("stencil,dtype,dw", [("25c", "f64", 16), ("25v", "f64", 8), ("25v", "f32", 16)])
def test_mwd_tiny_radius4(stencil, dtype, dw):
    u0, c, arr = inputs(stencil, 5, 3, 6, seed=4)
    got, _ = run_gpu(stencil, dtype, u0, c, arr, 3, algo="mwd", params={"diamond_width": dw})
    assert_bitwise(got, oracle_run(stencil, u0, c, arr, 3, dtype), "tiny %s %s" % (stencil, dtype))


@pytest.mark.parametrize("stencil", ["7c", "7v"])
def test_mwd_padded_layout(stencil):
    u0, c, arr = inputs(stencil, 50, 20, 9, seed=5)
    got, _ = run_gpu(stencil, "f64", u0, c, arr, 6, params={"diamond_width": 8}, pitch=(64, 25))
    assert_bitwise(got, oracle_run(stencil, u0, c, arr, 6), "padded")


def test_mwd_time_split_bitwise():
    import paper_1510_04995_amd as P
    from tests.gpu_util import torch_dev, upload
    torch, dev = torch_dev()
    u0, c, arr = inputs("7c", 90, 40, 16, seed=6)
    sw = P.Sweep("7c", "f64", 90, 40, 16, list(c), "mwd", {"diamond_width": 8})
    b0, b1 = upload(u0), upload(u0)
    out = sw.run(b0, b1, 5)
    other = b1 if out is b0 else b0
    out2 = sw.run(out, other, 6)
    whole = oracle_run("7c", u0, c, arr, 11)
    assert_bitwise(out2.cpu().numpy(), whole, "run(5); run(6) vs run(11)")
    sw.close()


def test_mwd_full_size_headline_vs_naive():
    """512^3 7-point constant, T = 64, in the benchmark's default launch
    configuration: MWD equals the GPU naive sweep and the oracle in every
    element (the oracle runs on the host's cores)."""
    import paper_1510_04995_amd as P
    from tests.gpu_util import torch_dev
    from workloads import WORKLOADS
    torch, dev = torch_dev()
    w = WORKLOADS["7pt-const-512"]
    u0, c, arr = inputs(w.stencil, w.nx, w.ny, w.nz, seed=0)
    g0 = torch.from_numpy(u0).to(dev)
    res = {}
    for algo in ("mwd", "naive"):
        sw = P.Sweep(w.stencil, "f64", w.nx, w.ny, w.nz, list(c), algo)
        b0, b1 = g0.clone(), g0.clone()
        res[algo] = sw.run(b0, b1, w.T)
        sw.close()
    rel, mx, nd = P.error_norms(res["mwd"], res["naive"], 1, w.nx, w.ny, w.nz)
    assert nd == 0 and mx == 0.0
    out = res["mwd"].cpu().numpy()
    naive = res["naive"].cpu().numpy()
    del res
    ref = oracle_run(w.stencil, u0, c, arr, w.T)
    assert_bitwise(out, ref, "MWD 512^3 vs oracle, whole grid")
    assert_bitwise(naive, ref, "naive 512^3 vs oracle, whole grid")


def test_small_workload_exact():
    """The 64^3, T = 16 workload: the naive sweep and the blocked sweep (in
    their default launch configurations) equal the oracle bit for bit."""
    from workloads import WORKLOADS
    w = WORKLOADS["7pt-const-64"]
    assert (w.nx, w.ny, w.nz, w.T) == (64, 64, 64, 16)
    u0, c, arr = inputs(w.stencil, w.nx, w.ny, w.nz, seed=0)
    ref = oracle_run(w.stencil, u0, c, arr, w.T)
    for algo in ("naive", "mwd"):
        got, _ = run_gpu(w.stencil, "f64", u0, c, arr, w.T, algo=algo)
        assert_bitwise(got, ref, "64^3 %s vs oracle" % algo)


@pytest.mark.parametrize("stencil,dtype,params", [("7c", "f64", {"variant": 1}),
                                                  ("7c", "f64", {"variant": 1, "diamond_width": 12, "threads_x": 128,
                                                                 "tile_x": 86}),
                                                  ("25c", "f64", {"variant": 1}),
                                                  ("7c", "f64", {"variant": 2}),
                                                  ("7c", "f64", {"variant": 3}),
                                                  ("7c", "f32", {"variant": 2})])
def test_full_size_dependency_driven(stencil, dtype, params):
    """512^3 (T = 64 for 7-point, 32 for 25-point) with the dependency-driven
    schedule, default shape (and, for 7-point, six x chunks per row), and
    with relaxed synchronisation: the whole grid equals the oracle (of the
    plan's precision)."""
    import paper_1510_04995_amd as P
    from tests.gpu_util import torch_dev
    from workloads import WORKLOADS
    torch, dev = torch_dev()
    w = WORKLOADS["7pt-const-512" if stencil == "7c" else "25pt-const-512"]
    u0, c, arr = inputs(w.stencil, w.nx, w.ny, w.nz, seed=0)
    g0 = torch.from_numpy(u0.astype(np.float64 if dtype == "f64" else np.float32)).to(dev)
    sw = P.Sweep(w.stencil, dtype, w.nx, w.ny, w.nz, [float(x) for x in c], "mwd", params)
    b0, b1 = g0.clone(), g0.clone()
    print("full size sweep", stencil, dtype, params, flush=True)
    out = sw.run(b0, b1, w.T)
    sw.check()
    got = out.cpu().numpy()
    sw.close()
    del b0, b1, g0, out
    assert_bitwise(got, oracle_run(w.stencil, u0, c, arr, w.T, dtype), "full size sweep %s %s %s"
                   % (stencil, dtype, params))


@pytest.mark.parametrize("stencil,dtype,n,T", [("7c", "f64", (509, 511, 513), 63), ("7c", "f32", (509, 511, 513), 63),
                                                ("25c", "f64", (509, 511, 513), 33)])
def test_mwd_odd_size_twin(stencil, dtype, n, T):
    """Odd-size twins of the benchmark grids (509 x 511 x 513, T = H*k + 3 for
    the default diamond heights H = 6 and 2) in the default launch
    configuration: ragged x chunks, partial diamonds at both y ends and
    clipped first and last rows at full scale.  The blocked sweep equals the
    naive GPU sweep and the oracle in every element."""
    import paper_1510_04995_amd as P
    from tests.gpu_util import torch_dev
    torch, dev = torch_dev()
    nx, ny, nz = n
    h = 1 if stencil == "7c" else 4
    u0, c, arr = inputs(stencil, nx, ny, nz, seed=5)
    npdt = np.float64 if dtype == "f64" else np.float32
    g0 = torch.from_numpy(u0.astype(npdt)).to(dev)
    res = {}
    for algo in ("mwd", "naive"):
        print("odd twin", stencil, dtype, n, T, algo, flush=True)
        sw = P.Sweep(stencil, dtype, nx, ny, nz, [float(x) for x in c], algo)
        b0, b1 = g0.clone(), g0.clone()
        res[algo] = sw.run(b0, b1, T)
        torch.cuda.synchronize()
        sw.close()
    rel, mx, nd = P.error_norms(res["mwd"], res["naive"], h, nx, ny, nz)
    assert nd == 0 and mx == 0.0
    out = res["mwd"].cpu().numpy()
    del res, g0
    assert_bitwise(out, oracle_run(stencil, u0, c, arr, T, dtype), "odd twin %s %s vs oracle, whole grid" % (stencil, dtype))


@pytest.mark.parametrize("name,dtype", [("25pt-const-512", "f64"), ("25pt-var-384", "f64"), ("25pt-var-384", "f32"),
                                        ("7pt-var-256x512x1024", "f64"), ("7pt-var-256x512x1024", "f32"),
                                        ("25pt-leapfrog-512", "f64"), ("25pt-leapfrog-512", "f32"),
                                        ("27pt-box-512", "f64"), ("27pt-box-512", "f32"),
                                        ("25pt-const-512", "f32"), ("7pt-const-512", "f32")])
def test_full_size_workloads(name, dtype):
    """The workloads at their full sizes in their default launch
    configurations (in FP32 the naive sweeps of the 7-point, 25-point and box
    stencils are register columns): the blocked and the naive sweep equal
    the oracle (same precision) in every element."""
    import paper_1510_04995_amd as P
    from tests.gpu_util import torch_dev
    from workloads import WORKLOADS
    torch, dev = torch_dev()
    w = WORKLOADS[name]
    h = w.radius
    u0, c, arr = inputs(w.stencil, w.nx, w.ny, w.nz, seed=0)
    npdt = np.float64 if dtype == "f64" else np.float32
    g0 = torch.from_numpy(u0.astype(npdt)).to(dev)
    coefs = [] if arr is None else [torch.from_numpy(a.astype(npdt)).to(dev) for a in arr]
    consts = None if c is None else [float(x) for x in c]
    algos = ("mwd", "naive")
    res = {}
    for algo in algos:
        print("full size", name, dtype, algo, flush=True)
        sw = P.Sweep(w.stencil, dtype, w.nx, w.ny, w.nz, consts, algo)
        b0, b1 = g0.clone(), g0.clone()
        res[algo] = sw.run(b0, b1, w.T, coefs)
        torch.cuda.synchronize()
        sw.close()
    if "mwd" in res:
        rel, mx, nd = P.error_norms(res["mwd"], res["naive"], h, w.nx, w.ny, w.nz)
        assert nd == 0 and mx == 0.0
    outs = {k: v.cpu().numpy() for k, v in res.items()}
    del res, coefs, g0
    ref = oracle_run(w.stencil, u0, c, arr, w.T, dtype)
    for algo, got in outs.items():
        assert_bitwise(got, ref, "%s %s %s vs oracle, whole grid" % (name, dtype, algo))


@pytest.mark.parametrize("stencil,dw,vx,wx,n,T", [("7c", 8, 1, 2, (140, 37, 13), 9), ("7v", 8, 2, 1, (131, 29, 11), 7),
                                                  ("25c", 16, 1, 1, (120, 45, 19), 5),
                                                  ("7c", 8, 2, 1, (131, 29, 11), 7),
                                                  ("25v", 8, 2, 1, (290, 21, 17), 3),
                                                  ("25c", 8, 2, 1, (290, 21, 17), 3),
                                                  ("27b", 8, 1, 2, (140, 37, 13), 9)])
def test_mwd_nonzero_halo(stencil, dw, vx, wx, n, T):
    """Arbitrary fixed Dirichlet values (and a -0.0) in the halo take the general path."""
    u0, c, arr = inputs(stencil, *n, seed=8)
    h = 4 if stencil.startswith("25") else 1
    rng = np.random.default_rng(3)
    halo = np.ones(u0.shape, dtype=bool)
    halo[h:-h, h:-h, h:-h] = False
    u0 = u0.copy()
    u0[halo] = rng.random(int(halo.sum())) - 0.5
    u0[0, 0, 0] = -0.0
    got, _ = run_gpu(stencil, "f64", u0, c, arr, T, algo="mwd", params=mwd_params(dw, vx, wx))
    assert_bitwise(got, oracle_run(stencil, u0, c, arr, T), "nonzero halo %s" % stencil)
    got32, _ = run_gpu(stencil, "f32", u0, c, arr, T, algo="mwd", params=mwd_params(dw, vx, wx))
    assert_bitwise(got32, oracle_run(stencil, u0, c, arr, T, "f32"), "nonzero halo f32 %s" % stencil)


def test_mwd_box_thin_grids_and_random_shapes():
    """The blocked box stencil on grids thinner than a diamond, a z-slab or
    the two-plane level skew, then on seeded random grids and step counts in
    every compiled shape: equal to the oracle bit for bit."""
    for dtype in ("f64", "f32"):
        for n in ((1, 1, 1), (9, 5, 3), (33, 7, 2), (130, 3, 1), (70, 1, 4)):
            u0, c, arr = inputs("27b", *n, seed=17)
            print("mwd box thin", dtype, n, flush=True)
            got, _ = run_gpu("27b", dtype, u0, c, arr, 6, algo="mwd")
            assert_bitwise(got, oracle_run("27b", u0, c, arr, 6, dtype), "box thin %s %s" % (dtype, n))
    rng = np.random.default_rng(27)
    for case in range(24):
        dtype = ("f64", "f32")[case % 2]
        dw = 8 if dtype == "f64" else (8, 12)[(case // 2) % 2]
        n = (int(rng.integers(1, 200)), int(rng.integers(1, 50)), int(rng.integers(1, 24)))
        T = int(rng.integers(0, 3 * dw))
        print("mwd box random", case, dtype, dw, n, T, flush=True)
        u0, c, arr = inputs("27b", *n, seed=100 + case)
        got, _ = run_gpu("27b", dtype, u0, c, arr, T, algo="mwd", params=mwd_params(dw, 1, 2))
        assert_bitwise(got, oracle_run("27b", u0, c, arr, T, dtype), "box random %d" % case)


def test_mwd_random_shapes_match_naive():
    """Seeded random grids, step counts and registered blocked shapes, all
    wavefront depths included (FP64 and FP32, both constant-coefficient
    stencils): the blocked sweep equals the naive GPU sweep bit for bit, and
    every tenth case also the oracle."""
    import paper_1510_04995_amd as P
    rng = np.random.default_rng(2024)
    shapes = {}
    for st in ("7c", "25c"):
        for dt in ("f64", "f32"):
            p = P.Sweep(st, dt, 64, 64, 64, [0.4, 0.1] if st == "7c" else [0.2, 0.05, 0.04, 0.03, 0.0133], "mwd")
            shapes[(st, dt)] = sorted({(q["diamond_width"], q["cells_per_lane"], q["threads_x"] // 64,
                                        q["wavefront_depth"], q["variant"]) for q in p.candidates()})
            p.close()
    for case in range(120):
        st = ("7c", "25c")[case % 2]
        dt = ("f64", "f32")[(case // 2) % 2]
        dw, vx, wx, nf, var = shapes[(st, dt)][rng.integers(len(shapes[(st, dt)]))]
        n = (int(rng.integers(1, 260)), int(rng.integers(1, 70)), int(rng.integers(1, 30)))
        T = int(rng.integers(0, 3 * dw))
        print("random", case, st, dt, dw, vx, wx, nf, var, n, T, flush=True)
        u0, c, arr = inputs(st, *n, seed=case)
        got, _ = run_gpu(st, dt, u0, c, arr, T, algo="mwd", params=dict(mwd_params(dw, vx, wx, 0, nf), variant=var),
                         check=var != 0)
        naive, _ = run_gpu(st, dt, u0, c, arr, T, algo="naive")
        assert_bitwise(got, naive, "random case %d %s %s Dw=%d vx=%d wx=%d nf=%d variant=%d n=%s T=%d"
                       % (case, st, dt, dw, vx, wx, nf, var, n, T))
        if case % 10 == 0:
            assert_bitwise(got, oracle_run(st, u0, c, arr, T, dt), "random case %d vs oracle" % case)
