"""Helpers shared by the GPU tests: upload seeded inputs, run a plan, download."""
import numpy as np

from workloads import field_and_coefs, RADIUS


def torch_dev():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a visible MI355X")
    return torch, torch.device("cuda:0")


def upload(a, pitch_x=None, pitch_y=None, h=None):
    """numpy (nz+2h, ny+2h, nx+2h) -> contiguous device tensor in padded layout."""
    torch, dev = torch_dev()
    if pitch_x is None and pitch_y is None:
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    nzp, nyp, nxp = a.shape
    py = pitch_y or nyp
    px = pitch_x or nxp
    t = torch.full((nzp, py, px), float("nan"), dtype=torch.from_numpy(a[:1, :1, :1].copy()).dtype, device=dev)
    t[:, :nyp, :nxp] = torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    return t


def run_gpu(stencil, dtype, u0, consts, arrays, T, algo="mwd", params=None, poison=True, pitch=None,
            return_tensors=False, prev=None, check=False):
    """Run the library on seeded numpy inputs; returns the unpadded numpy result.

    buf1 starts as a copy of u0 whose interior is NaN (``poison``: the
    first-order stencils must not read it), except for the second-order-in-time
    stencil, which reads it as u^{-1}: ``prev`` (default u0)."""
    import paper_1510_04995_amd as P
    torch, dev = torch_dev()
    h = RADIUS[stencil]
    nzp, nyp, nxp = u0.shape
    nz, ny, nx = nzp - 2 * h, nyp - 2 * h, nxp - 2 * h
    px, py = (pitch or (None, None))
    npdt = np.float64 if dtype == "f64" else np.float32
    b0 = upload(u0.astype(npdt), px, py)
    if stencil == "25l":
        b1 = upload((u0 if prev is None else prev).astype(npdt), px, py)
    else:
        b1 = b0.clone()
        if poison:
            b1[h:h + nz, h:h + ny, h:h + nx] = float("nan")
    coefs = [upload(a.astype(npdt), px, py) for a in (arrays or [])]
    sw = P.Sweep(stencil, dtype, nx, ny, nz, None if consts is None else [float(c) for c in consts], algo, params,
                 pitch_x=px or 0, pitch_y=py or 0)
    out = sw.run(b0, b1, T, coefs)
    torch.cuda.synchronize()
    if check:
        sw.check()   # no dependency wait gave up
    res = out[:, :nyp, :nxp].cpu().numpy()
    info = sw.info()
    sw.close()
    if return_tensors:
        return res, info, (b0, b1, out)
    return res, info


def oracle_run(stencil, u0, consts, arrays, T, dtype="f64", prev=None):
    from oracle import sweep as osw
    npdt = np.float64 if dtype == "f64" else np.float32
    b0 = np.ascontiguousarray(u0.astype(npdt))
    b1 = b0.copy() if prev is None else np.ascontiguousarray(prev.astype(npdt))
    ar = None if arrays is None else [np.ascontiguousarray(a.astype(npdt)) for a in arrays]
    c = None if consts is None else np.asarray(consts, dtype=npdt)
    idx = osw.sweep(stencil, b0, b1, T, c, ar)
    return (b0, b1)[idx]


def inputs(stencil, nx, ny, nz, seed=0):
    return field_and_coefs(stencil, nx, ny, nz, seed=seed)
