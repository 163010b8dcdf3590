"""girih_run_noalloc (fixed device scratch, no allocation) against girih_run,
through the C ABI: two calls in a row on one device, the second on a smaller
grid, bit for bit; the blocked sweep of a constant- and a variable-coefficient
stencil, with relaxed synchronisation (whose error word sits in the fixed
array too), the second-order stencil (whose u^{-1} a run may copy into
the fixed pair) and the box stencil (three-plane stage rows); a grid over
the fixed limit is refused before any launch."""
import numpy as np
import pytest

import paper_1510_04995_amd.girih as G
from tests.gpu_util import inputs, torch_dev, upload

pytestmark = pytest.mark.gpu


def run_both(stencil, dtype, n, T, params):
    """(result of girih_run, result of girih_run_noalloc) on the same inputs."""
    torch, dev = torch_dev()
    h = G.RADIUS[stencil]
    u0, c, arr = inputs(stencil, *n, seed=31)
    npdt = np.float64 if dtype == "f64" else np.float32
    grid = G.make_grid(*n, h)
    plan = G.girih_plan(stencil, dtype, grid, None if c is None else [float(x) for x in c], "mwd", params)
    coefs = [upload(a.astype(npdt)) for a in (arr or [])]
    stream = torch.cuda.current_stream().cuda_stream
    out = []
    prev = None
    if stencil == "25l":   # u^{-1}: u^0's halo, a random interior
        prev = u0.copy()
        prev[h:-h, h:-h, h:-h] = np.random.default_rng(32).random(tuple(d - 2 * h for d in u0.shape))
    for fn in (G.girih_run, G.girih_run_noalloc):
        b0 = upload(u0.astype(npdt))
        if prev is None:
            b1 = b0.clone()
            b1[h:-h, h:-h, h:-h] = float("nan")
        else:
            b1 = upload(prev.astype(npdt))
        print(fn.__name__, stencil, dtype, n, T, flush=True)
        idx = fn(plan, b0.data_ptr(), b1.data_ptr(), [t.data_ptr() for t in coefs], T, stream)
        torch.cuda.synchronize()
        out.append((b0, b1)[idx].cpu().numpy())
    G.girih_destroy(plan)
    return out


@pytest.mark.parametrize("stencil,dtype,params", [("7c", "f64", {"diamond_width": 8}),
                                                  ("7v", "f32", {"diamond_width": 12}),
                                                  ("7c", "f64", {"variant": 2}),
                                                  ("25l", "f64", {}),
                                                  ("27b", "f32", {})])
def test_noalloc_equals_run_twice_second_smaller(stencil, dtype, params):
    for n, T in (((150, 61, 23), 11), ((70, 29, 9), 6)):
        ref, got = run_both(stencil, dtype, n, T, params)
        assert np.array_equal(ref, got), (stencil, dtype, n, T)


def test_noalloc_refuses_a_grid_over_the_limit():
    torch, dev = torch_dev()
    # 260^3 FP64 with its halo is 140 MB per array: over the 64 MiB limit
    grid = G.make_grid(260, 260, 260, 1)
    plan = G.girih_plan("7c", "f64", grid, (0.4, 0.1), "mwd")
    with pytest.raises(G.GirihError) as e:
        G.girih_run_noalloc(plan, 4096, 8192, [], 3, 0)   # refused before the pointers are used
    assert e.value.code == G.E_SCRATCH
    G.girih_destroy(plan)
