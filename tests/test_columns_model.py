"""Host-side model of the naive register-column kernels' index logic
(naive_box_cols_kernel: box stencil, variant 1; naive_star_cols_kernel:
constant-coefficient star stencils, variant 2).

It re-derives, in numpy, how the host sizes the grid (x blocks of 64 - 2R
stored cells, y blocks of W x KY rows, z chunks) and how each block, wave
and lane of the kernel forms its rows, columns and planes, and checks over
many small and ragged configurations:

* bounds: every load (rows and side rows clamped into the haloed box, the
  lane's column clamped likewise, planes z0 - R .. z1 - 1 + R) lies inside
  the padded array, for zero chunk remainders and ragged ones;
* coverage: every interior cell is stored exactly once, by a lane whose x
  neighbours x - r .. x + r (r <= R) are held, unclamped, by lanes of the
  same wave (the DPP moves reach them) and whose y and z neighbours are
  rows and planes the wave loaded for that step;
* the XCD-contiguous block numbering is a permutation of the blocks.

They need no GPU; the GPU parity tests check the kernels themselves.
"""
import numpy as np
import pytest


def xcd_runs(nb, on=True):
    """Block index each launch-order id sweeps (the kernels' renumbering)."""
    nx = 8 if on else 1
    lid = np.arange(nb)
    per, extra = nb // nx, nb % nx
    xcd, pos = lid % nx, lid // nx
    return np.where(xcd < extra, xcd * (per + 1), extra * (per + 1) + (xcd - extra) * per) + pos


def model(R, nx, ny, nz, W, KY, tz, box, plant=False):
    """Loads and stores of one launch: returns (load rows/cols/planes, store
    (z, y, x) list, neighbour checks failed).  ``plant``: lane R - 1 also
    stores (a mistake the checks must catch)."""
    own = 64 - 2 * R
    gx, gy, gz = -(-nx // own), -(-ny // (W * KY)), -(-nz // tz)
    nb = gx * gy * gz
    run = xcd_runs(nb)
    assert sorted(run.tolist()) == list(range(nb))
    stores = []
    bad = 0
    lo = {"y": 1 << 60, "x": 1 << 60, "z": 1 << 60}
    hi = {"y": -(1 << 60), "x": -(1 << 60), "z": -(1 << 60)}

    def seen(k, v):
        lo[k] = min(lo[k], int(np.min(v)))
        hi[k] = max(hi[k], int(np.max(v)))

    lane = np.arange(64)
    for t in run:
        bx, by, bz = t % gx, (t // gx) % gy, t // (gx * gy)
        z0 = bz * tz
        z1 = min(z0 + tz, nz)
        if z0 >= z1:
            continue
        for wave in range(W):
            y0 = (by * W + wave) * KY
            if y0 >= ny:
                continue
            x = bx * own + lane - R
            xc = np.minimum(np.maximum(x, -R), nx + R - 1)
            seen("x", xc)
            if box:
                rows = [min(y0 - 1 + r, ny) for r in range(KY + 2)]
            else:
                clampy = lambda y: max(-R, min(y, ny + R - 1))
                rows = [clampy(y0 + k) for k in range(KY)] + \
                       [clampy(y0 - R + i) for i in range(R)] + [clampy(y0 + KY + i) for i in range(R)]
            seen("y", np.array(rows))
            seen("z", np.array([z0 - R, z1 - 1 + R]))
            st_x = (lane >= (R - 1 if plant else R)) & (lane < 64 - R) & (x < nx)
            for k in range(KY):
                y = y0 + k
                if y >= ny:
                    continue
                for z in range(z0, z1):
                    for ln in np.nonzero(st_x)[0]:
                        stores.append((z, y, int(x[ln])))
                        # x neighbours: lanes ln +- r hold columns x +- r unclamped
                        for r in range(1, R + 1):
                            if not (0 <= ln - r and ln + r < 64 and xc[ln + r] == x[ln] + r
                                    and xc[ln - r] == x[ln] - r):
                                bad += 1
                # y neighbours of row y within the loaded rows, unclamped
                need = range(y - R, y + R + 1)
                held = set(rows)
                if any(v not in held for v in need):
                    bad += 1
    return lo, hi, stores, bad


CASES = [
    # (R, nx, ny, nz, W, KY, tz, box)
    (1, 130, 47, 12, 2, 8, 32, True), (1, 61, 5, 9, 4, 2, 7, True), (1, 62, 16, 3, 2, 4, 200, True),
    (1, 63, 17, 4, 4, 8, 41, True), (1, 1, 1, 1, 2, 2, 12, True), (1, 124, 1, 2, 4, 4, 5, True),
    (1, 70, 33, 41, 2, 8, 7, False), (1, 62, 16, 3, 4, 2, 5, False), (1, 63, 9, 5, 2, 4, 12, False),
    (4, 55, 9, 7, 2, 8, 5, False), (4, 56, 16, 3, 4, 2, 41, False), (4, 57, 17, 4, 2, 4, 12, False),
    (4, 1, 1, 1, 2, 8, 12, False), (4, 130, 47, 12, 4, 8, 5, False), (4, 3, 5, 1, 2, 2, 7, False),
]


@pytest.mark.parametrize("R,nx,ny,nz,W,KY,tz,box", CASES)
def test_register_columns_bounds_and_coverage(R, nx, ny, nz, W, KY, tz, box):
    lo, hi, stores, bad = model(R, nx, ny, nz, W, KY, tz, box)
    # every load inside the haloed box [-R, n + R)
    assert lo["x"] >= -R and hi["x"] <= nx + R - 1
    assert lo["y"] >= -R and hi["y"] <= ny + R - 1
    assert lo["z"] >= -R and hi["z"] <= nz + R - 1
    # every interior cell stored exactly once
    assert len(stores) == nx * ny * nz
    assert len(set(stores)) == nx * ny * nz
    assert bad == 0


def test_random_shapes():
    rng = np.random.default_rng(11)
    for _ in range(25):
        box = bool(rng.integers(2))
        R = 1 if box else int(rng.choice([1, 4]))
        n = (int(rng.integers(1, 140)), int(rng.integers(1, 40)), int(rng.integers(1, 14)))
        W, KY, tz = int(rng.choice([2, 4])), int(rng.choice([2, 4, 8])), int(rng.integers(1, 20))
        lo, hi, stores, bad = model(R, *n, W, KY, tz, box)
        assert lo["x"] >= -R and hi["x"] <= n[0] + R - 1 and lo["y"] >= -R and hi["y"] <= n[1] + R - 1
        assert lo["z"] >= -R and hi["z"] <= n[2] + R - 1
        assert len(stores) == len(set(stores)) == n[0] * n[1] * n[2] and bad == 0


def test_a_planted_extra_lane_is_caught():
    """With one more storing lane per wave (lane R - 1, whose x - R
    neighbour is in no lane) the model reports missing neighbours and
    cells stored twice."""
    for R, box in ((1, True), (1, False), (4, False)):
        lo, hi, stores, bad = model(R, 130, 9, 3, 2, 4, 5, box, plant=True)
        assert bad > 0 and len(stores) > len(set(stores))
