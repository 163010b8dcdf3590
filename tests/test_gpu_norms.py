"""The library's FP64 error reduction (girih_error_norms), on which the
full-size parity checks rest, against numpy on the host: planted one-ulp
flips, a NaN, a -0.0 against +0.0, halo differences that must not count, and
an FP32-against-FP64 pair.  Through the C ABI."""
import numpy as np
import pytest

import paper_1510_04995_amd.girih as G

pytestmark = pytest.mark.gpu


def norms(a, b, h, nx, ny, nz):
    """Raw out[4] of girih_error_norms for two host arrays of the padded layout."""
    from tests.gpu_util import torch_dev
    torch, dev = torch_dev()
    ta, tb = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    grid = G.make_grid(nx, ny, nz, h, a.shape[2], a.shape[1])
    name = {np.dtype(np.float64): "f64", np.dtype(np.float32): "f32"}
    return G.girih_error_norms(grid, name[a.dtype], ta.data_ptr(), name[b.dtype], tb.data_ptr(),
                               torch.cuda.current_stream().cuda_stream)


def host_norms(a, b, h, nx, ny, nz):
    core = (slice(h, h + nz), slice(h, h + ny), slice(h, h + nx))
    x, y = a[core].astype(np.float64), b[core].astype(np.float64)
    d = x - y
    return np.sqrt(np.sum(d * d)), np.sqrt(np.sum(y * y)), np.max(np.abs(d)), core


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_planted_differences(dtype):
    nx, ny, nz, h = 37, 29, 23, 1
    rng = np.random.default_rng(12)
    b = (rng.random((nz + 2 * h, ny + 2 * h + 3, nx + 2 * h + 5)) - 0.5).astype(dtype)   # padded pitches
    a = b.copy()
    out = norms(a, b, h, nx, ny, nz)
    assert out[0] == 0 and out[2] == 0 and out[3] == 0
    # differences in the halo and in the pitch padding are not counted
    a[0, 5, 5] += 1
    a[4, ny + 2 * h + 1, 3] = np.nan
    a[4, 3, nx + 2 * h + 2] = 7
    out = norms(a, b, h, nx, ny, nz)
    assert out[0] == 0 and out[2] == 0 and out[3] == 0
    # one ulp at two interior points, a signed zero
    p1, p2, p3 = (1, 1, 1), (nz, ny, nx), (12, 7, 30)
    a[p1] = np.nextafter(b[p1], dtype(np.inf))
    a[p2] = np.nextafter(b[p2], dtype(-np.inf))
    b[p3] = dtype(0.0)
    a[p3] = dtype(-0.0)
    out = norms(a, b, h, nx, ny, nz)
    d2, b2, mx, _ = host_norms(a, b, h, nx, ny, nz)
    assert out[3] == 3
    assert out[2] == mx and mx > 0
    assert out[0] == pytest.approx(d2, rel=1e-14)
    assert out[1] == pytest.approx(b2, rel=1e-14)
    # a NaN anywhere in the interior shows in the difference norm and the max
    a[(5, 20, 9)] = np.nan
    out = norms(a, b, h, nx, ny, nz)
    assert np.isnan(out[0]) and np.isnan(out[2]) and out[3] == 4


def test_f32_against_f64():
    nx, ny, nz, h = 41, 17, 19, 4
    rng = np.random.default_rng(13)
    b = rng.random((nz + 2 * h, ny + 2 * h, nx + 2 * h))
    a = b.astype(np.float32)
    out = norms(a, b, h, nx, ny, nz)
    d2, b2, mx, _ = host_norms(a, b, h, nx, ny, nz)
    assert out[0] == pytest.approx(d2, rel=1e-12) and d2 > 0
    assert out[1] == pytest.approx(b2, rel=1e-14)
    assert out[2] == mx
    # the other argument order
    out2 = norms(b, a, h, nx, ny, nz)
    d2b, b2b, mxb, _ = host_norms(b, a, h, nx, ny, nz)
    assert out2[0] == pytest.approx(d2b, rel=1e-12) and out2[2] == mxb
    assert out2[1] == pytest.approx(b2b, rel=1e-14)
