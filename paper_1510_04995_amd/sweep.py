"""PyTorch-facing wrapper of one plan: device memory and streams from torch,
all computation in ``libgirih.so``.

Tensors are C-contiguous CUDA (HIP) tensors of shape (nz+2h, pitch_y, pitch_x)
in float64 or float32; element (k, j, i) of the paper's U[k][j][i] (x fastest)
sits at [k+h, j+h, i+h].
"""
from . import girih as G


def _dtype_name(t):
    import torch
    if t.dtype == torch.float64:
        return "f64"
    if t.dtype == torch.float32:
        return "f32"
    raise TypeError("grid tensors must be float64 or float32")


class Sweep:
    """A plan for ``T`` steps of one stencil ("7c", "7v", "25c", "25v", "25l", "27b") on one grid.

    ``algo``: "mwd" (diamond rows, wavefront along z; "7c" and "25c") or "naive".
    ``params``: dict of ``girih_params`` fields (zeros take defaults).
    """

    def __init__(self, stencil, dtype, nx, ny, nz, const_coefs=None, algo="mwd", params=None,
                 pitch_x=0, pitch_y=0):
        self.stencil, self.dtype, self.algo = stencil, dtype, algo
        self.h = G.RADIUS[stencil]
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.grid = G.make_grid(nx, ny, nz, self.h, pitch_x, pitch_y)
        self.plan = G.girih_plan(stencil, dtype, self.grid, const_coefs, algo, params)
        self.pitch_x = pitch_x or self.nx + 2 * self.h
        self.pitch_y = pitch_y or self.ny + 2 * self.h

    @property
    def shape(self):
        return (self.nz + 2 * self.h, self.pitch_y, self.pitch_x)

    def _check(self, t, what):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError("%s must be a CUDA (HIP) tensor" % what)
        if not t.is_contiguous() or tuple(t.shape) != self.shape:
            raise ValueError("%s must be contiguous with shape %s" % (what, self.shape))
        if _dtype_name(t) != self.dtype:
            raise TypeError("%s has the wrong dtype for a %s plan" % (what, self.dtype))

    def run(self, buf0, buf1, T, coefs=(), stream=None):
        """Run T steps; returns the tensor (buf0 or buf1) that holds u^T.

        ``buf0`` holds u^0 with its halo, ``buf1`` the same halo; for the
        second-order-in-time stencil "25l" the interior of ``buf1`` is read as
        u^{-1} (a copy of u^0 starts from rest).  Both buffers are clobbered;
        the other one returns u^{T-1} for "25l"."""
        import torch
        self._check(buf0, "buf0")
        self._check(buf1, "buf1")
        coefs = list(coefs or ())
        if len(coefs) != G.N_COEF[self.stencil]:
            raise ValueError("stencil %s takes %d coefficient arrays" % (self.stencil, G.N_COEF[self.stencil]))
        for m, c in enumerate(coefs):
            self._check(c, "coefs[%d]" % m)
        s = stream if stream is not None else torch.cuda.current_stream()
        idx = G.girih_run(self.plan, buf0.data_ptr(), buf1.data_ptr(), [c.data_ptr() for c in coefs], T,
                          s.cuda_stream)
        return (buf0, buf1)[idx]

    def tune(self, mode="hillclimb", T=64, max_seconds=30.0, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        return G.girih_tune(self.plan, mode, T, max_seconds, s.cuda_stream)

    def set_candidates(self, cands):
        G.girih_tune_set_candidates(self.plan, cands)

    def candidates(self):
        return G.girih_candidates(self.plan)

    def tune_log(self):
        return G.girih_tune_log(self.plan)

    def info(self):
        params, lds, bpl = G.girih_plan_info(self.plan)
        return {"params": params, "lds_bytes": lds, "model_bytes_per_lup": bpl}

    def set_timing(self, enable=True):
        """Bracket every sweep-kernel launch of later runs with HIP events."""
        G.girih_set_timing(self.plan, enable)

    def timing(self):
        """(launches, total kernel milliseconds) of the most recent run."""
        return G.girih_timing(self.plan)

    def check(self, stream=None):
        """Synchronise; raise (E_STALL) if a bounded device wait of the last
        run (variants 1-3) gave up."""
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        G.girih_check(self.plan, s.cuda_stream)

    def set_lds_budget(self, nbytes):
        """Prune tuner candidates whose workgroup needs more LDS (0: none)."""
        G.girih_set_lds_budget(self.plan, nbytes)

    def set_wait_limit(self, polls):
        G.girih_set_wait_limit(self.plan, polls)

    def set_params(self, params):
        G.girih_plan_set_params(self.plan, params)

    def close(self):
        if getattr(self, "plan", None):
            G.girih_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def error_norms(a, b, h, nx, ny, nz, stream=None):
    """(rel_l2, max_abs, n_bitwise_different) of a against b, in float64, on the GPU."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    grid = G.make_grid(nx, ny, nz, h, a.shape[2], a.shape[1])
    d2, b2, mx, nd = G.girih_error_norms(grid, _dtype_name(a), a.data_ptr(), _dtype_name(b), b.data_ptr(),
                                         s.cuda_stream)
    return (d2 / b2 if b2 > 0 else d2), mx, int(nd)
