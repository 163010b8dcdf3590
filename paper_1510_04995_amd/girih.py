"""ctypes binding of ``libgirih.so`` (declared in ``include/girih.h``).

Argument marshalling only: every step of the sweep runs in the library's HIP
kernels.  Device memory and streams come from PyTorch (``tensor.data_ptr()``,
``torch.cuda.current_stream().cuda_stream``).  If the library is missing this
module raises on first use — there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgirih.so")

OK = 0
E_INVALID, E_UNSUPPORTED, E_LDS, E_HIP, E_NOMEM, E_NOGPU, E_SCRATCH, E_STALL = -1, -2, -3, -4, -5, -6, -7, -8

STENCIL_IDS = {"7c": 0, "7v": 1, "25c": 2, "25v": 3, "25l": 4, "27b": 5}
DTYPE_IDS = {"f64": 0, "f32": 1}
ALGO_IDS = {"naive": 0, "mwd": 1}
TUNE_MODES = {"exhaustive": 0, "hillclimb": 1, "model": 2}
RADIUS = {"7c": 1, "7v": 1, "25c": 4, "25v": 4, "25l": 4, "27b": 1}
N_COEF = {"7c": 0, "7v": 7, "25c": 0, "25v": 13, "25l": 1, "27b": 0}


class GirihGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("halo", ctypes.c_int32), ("pitch_x", ctypes.c_int64), ("pitch_y", ctypes.c_int64)]


class GirihParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("diamond_width", "wavefront_depth", "tile_x", "tile_y",
                                                "tile_z", "threads_x", "threads_y", "variant",
                                                "cells_per_lane")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}

    @classmethod
    def from_dict(cls, d):
        p = cls()
        for n, _ in cls._fields_:
            setattr(p, n, int(d.get(n, 0) or 0))
        return p


class GirihTuneRecord(ctypes.Structure):
    _fields_ = [("params", GirihParams), ("lds_bytes", ctypes.c_int64), ("steps", ctypes.c_int64),
                ("seconds", ctypes.c_double), ("glups", ctypes.c_double), ("repeats", ctypes.c_int32),
                ("status", ctypes.c_int32)]


class GirihError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (what, _lib().girih_strerror(code).decode(), code))


_LIB = None

MEASURE_FN = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.POINTER(GirihParams), ctypes.c_void_p)
TIME_FN = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.c_int64, ctypes.c_void_p)

# name -> (restype, argtypes): the exported symbols of include/girih.h
SIGNATURES = {
    "girih_plan": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(GirihGrid), ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                  ctypes.POINTER(GirihParams)]),
    "girih_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_int64,
                                 ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "girih_run_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_int64,
                                         ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "girih_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                  ctypes.c_void_p, ctypes.POINTER(GirihParams), ctypes.POINTER(ctypes.c_double)]),
    "girih_tune_set_candidates": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(GirihParams), ctypes.c_int32]),
    "girih_tune_search": (ctypes.c_int, [ctypes.POINTER(GirihParams), ctypes.c_int32, ctypes.c_int32, MEASURE_FN,
                                         ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]),
    "girih_adaptive_time": (ctypes.c_int, [TIME_FN, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]),
    "girih_candidates": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(GirihParams), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32)]),
    "girih_tune_log": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(GirihTuneRecord), ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_int32)]),
    "girih_plan_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(GirihParams),
                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]),
    "girih_plan_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(GirihParams)]),
    "girih_set_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "girih_set_wait_limit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32]),
    "girih_set_lds_budget": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "girih_check": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "girih_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "girih_destroy": (None, [ctypes.c_void_p]),
    "girih_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "girih_error_norms": (ctypes.c_int, [ctypes.POINTER(GirihGrid), ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "girih_version": (ctypes.c_char_p, []),
    "girih_mlp_param_count": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.POINTER(ctypes.c_int64)]),
    "girih_mlp_work_count": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_int64)]),
    "girih_mlp_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int64, ctypes.c_void_p]),
    "girih_mlp_loss_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "girih_mlp_adam": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_int64, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_int32, ctypes.c_void_p]),
}


def _lib():
    global _LIB
    if _LIB is None:
        # PyTorch ships its own HIP runtime under the same soname as the
        # system's; loading torch first makes the library bind to that one
        # runtime, so torch's device pointers and streams are valid in it.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libgirih.so is not built (run __graft_entry__.build() or "
                               "python paper_1510_04995_amd/build.py)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def _check(rc, what):
    if rc != OK:
        raise GirihError(rc, what)


def make_grid(nx, ny, nz, halo, pitch_x=0, pitch_y=0):
    return GirihGrid(int(nx), int(ny), int(nz), int(halo), int(pitch_x), int(pitch_y))


# ---- thin wrappers with the C names -------------------------------------------

def girih_plan(stencil, dtype, grid, const_coefs=None, algo="mwd", params=None):
    out = ctypes.c_void_p()
    cc = None
    if const_coefs is not None:
        vals = [float(c) for c in const_coefs]
        cc = (ctypes.c_double * len(vals))(*vals)
    p = None
    if params is not None:
        p = params if isinstance(params, GirihParams) else GirihParams.from_dict(params)
    rc = _lib().girih_plan(ctypes.byref(out), STENCIL_IDS[stencil], DTYPE_IDS[dtype], ctypes.byref(grid),
                           cc, ALGO_IDS[algo], ctypes.byref(p) if p is not None else None)
    _check(rc, "girih_plan")
    return out


def girih_run(plan, buf0_ptr, buf1_ptr, coef_ptrs, T, stream_ptr):
    n = len(coef_ptrs)
    arr = (ctypes.c_void_p * max(n, 1))(*[ctypes.c_void_p(int(q)) for q in coef_ptrs]) if n else None
    res = ctypes.c_int32(-1)
    rc = _lib().girih_run(plan, ctypes.c_void_p(int(buf0_ptr)), ctypes.c_void_p(int(buf1_ptr)),
                          ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p)) if n else None, n, int(T),
                          ctypes.c_void_p(int(stream_ptr)) if stream_ptr else None, ctypes.byref(res))
    _check(rc, "girih_run")
    return res.value


def girih_run_noalloc(plan, buf0_ptr, buf1_ptr, coef_ptrs, T, stream_ptr):
    """girih_run with the library's fixed device scratch (no allocation)."""
    n = len(coef_ptrs)
    arr = (ctypes.c_void_p * max(n, 1))(*[ctypes.c_void_p(int(q)) for q in coef_ptrs]) if n else None
    res = ctypes.c_int32(-1)
    rc = _lib().girih_run_noalloc(plan, ctypes.c_void_p(int(buf0_ptr)), ctypes.c_void_p(int(buf1_ptr)),
                                  ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p)) if n else None, n, int(T),
                                  ctypes.c_void_p(int(stream_ptr)) if stream_ptr else None, ctypes.byref(res))
    _check(rc, "girih_run_noalloc")
    return res.value


def girih_tune(plan, mode, T, max_seconds, stream_ptr):
    best = GirihParams()
    g = ctypes.c_double(0)
    rc = _lib().girih_tune(plan, TUNE_MODES[mode] if isinstance(mode, str) else int(mode), int(T),
                           float(max_seconds), ctypes.c_void_p(int(stream_ptr)) if stream_ptr else None,
                           ctypes.byref(best), ctypes.byref(g))
    _check(rc, "girih_tune")
    return best.as_dict(), g.value


def girih_tune_search(cands, mode, measure, max_seconds=1e9):
    """The tuner's search over `cands` (dicts) with a Python measurement
    measure(params_dict) -> GLUP/s; returns (best index, best GLUP/s, number
    of candidates measured)."""
    arr = (GirihParams * max(len(cands), 1))(*[GirihParams.from_dict(c) for c in cands])
    cb = MEASURE_FN(lambda p, ctx: float(measure(p.contents.as_dict())))
    bi, bg, nm = ctypes.c_int32(-1), ctypes.c_double(0), ctypes.c_int32(0)
    rc = _lib().girih_tune_search(arr, len(cands), TUNE_MODES[mode] if isinstance(mode, str) else int(mode), cb,
                                  None, float(max_seconds), ctypes.byref(bi), ctypes.byref(bg), ctypes.byref(nm))
    if rc != E_UNSUPPORTED:
        _check(rc, "girih_tune_search")
    return bi.value, bg.value, nm.value


def girih_adaptive_time(time_reps, tol=0.03, min_seconds=0.05, max_seconds=1e9, max_tries=12):
    """The tuner's adaptive test length with a Python timer time_reps(reps) ->
    seconds; returns (seconds per run, reps of the accepted measurement,
    measurements taken)."""
    cb = TIME_FN(lambda k, ctx: float(time_reps(int(k))))
    per, reps, tries = ctypes.c_double(0), ctypes.c_int64(0), ctypes.c_int32(0)
    _check(_lib().girih_adaptive_time(cb, None, float(tol), float(min_seconds), float(max_seconds), int(max_tries),
                                      ctypes.byref(per), ctypes.byref(reps), ctypes.byref(tries)),
           "girih_adaptive_time")
    return per.value, reps.value, tries.value


def girih_tune_set_candidates(plan, cands):
    arr = (GirihParams * max(len(cands), 1))(*[c if isinstance(c, GirihParams) else GirihParams.from_dict(c)
                                               for c in cands])
    _check(_lib().girih_tune_set_candidates(plan, arr, len(cands)), "girih_tune_set_candidates")


def girih_candidates(plan):
    n = ctypes.c_int32(0)
    _check(_lib().girih_candidates(plan, None, 0, ctypes.byref(n)), "girih_candidates")
    arr = (GirihParams * max(n.value, 1))()
    _check(_lib().girih_candidates(plan, arr, n.value, ctypes.byref(n)), "girih_candidates")
    return [arr[i].as_dict() for i in range(n.value)]


def girih_tune_log(plan):
    n = ctypes.c_int32(0)
    _check(_lib().girih_tune_log(plan, None, 0, ctypes.byref(n)), "girih_tune_log")
    arr = (GirihTuneRecord * max(n.value, 1))()
    _check(_lib().girih_tune_log(plan, arr, n.value, ctypes.byref(n)), "girih_tune_log")
    out = []
    for i in range(n.value):
        r = arr[i]
        out.append(dict(params=r.params.as_dict(), lds_bytes=r.lds_bytes, steps=r.steps, seconds=r.seconds,
                        glups=r.glups, repeats=r.repeats, status=r.status))
    return out


def girih_plan_info(plan):
    p = GirihParams()
    lds = ctypes.c_int64(0)
    bpl = ctypes.c_double(0)
    _check(_lib().girih_plan_info(plan, ctypes.byref(p), ctypes.byref(lds), ctypes.byref(bpl)), "girih_plan_info")
    return p.as_dict(), lds.value, bpl.value


def girih_plan_set_params(plan, params):
    p = params if isinstance(params, GirihParams) else GirihParams.from_dict(params)
    _check(_lib().girih_plan_set_params(plan, ctypes.byref(p)), "girih_plan_set_params")


def girih_set_lds_budget(plan, nbytes):
    _check(_lib().girih_set_lds_budget(plan, int(nbytes)), "girih_set_lds_budget")


def girih_set_wait_limit(plan, polls):
    _check(_lib().girih_set_wait_limit(plan, int(polls)), "girih_set_wait_limit")


def girih_check(plan, stream_ptr):
    """Synchronise the stream; GirihError(E_STALL) if a bounded device wait
    of the plan's last run (variants 1-3) gave up."""
    _check(_lib().girih_check(plan, ctypes.c_void_p(int(stream_ptr)) if stream_ptr else None), "girih_check")


def girih_set_timing(plan, enable):
    _check(_lib().girih_set_timing(plan, 1 if enable else 0), "girih_set_timing")


def girih_timing(plan):
    n = ctypes.c_int32(0)
    ms = ctypes.c_double(0)
    _check(_lib().girih_timing(plan, ctypes.byref(n), ctypes.byref(ms)), "girih_timing")
    return n.value, ms.value


def girih_destroy(plan):
    _lib().girih_destroy(plan)


def girih_strerror(code):
    return _lib().girih_strerror(int(code)).decode()


def girih_error_norms(grid, dtype_a, a_ptr, dtype_b, b_ptr, stream_ptr):
    out = (ctypes.c_double * 4)()
    rc = _lib().girih_error_norms(ctypes.byref(grid), DTYPE_IDS[dtype_a], ctypes.c_void_p(int(a_ptr)),
                                  DTYPE_IDS[dtype_b], ctypes.c_void_p(int(b_ptr)),
                                  ctypes.c_void_p(int(stream_ptr)) if stream_ptr else None, out)
    _check(rc, "girih_error_norms")
    return list(out)


def girih_version():
    return _lib().girih_version().decode()


def _vp(x):
    return ctypes.c_void_p(int(x)) if x else None


def girih_mlp_param_count(n_in, n_hidden, n_layers):
    c = ctypes.c_int64(0)
    _check(_lib().girih_mlp_param_count(n_in, n_hidden, n_layers, ctypes.byref(c)), "girih_mlp_param_count")
    return c.value


def girih_mlp_work_count(n_in, n_hidden, n_layers, n):
    c = ctypes.c_int64(0)
    _check(_lib().girih_mlp_work_count(n_in, n_hidden, n_layers, n, ctypes.byref(c)), "girih_mlp_work_count")
    return c.value


def girih_mlp_forward(params, n_in, n_hidden, n_layers, x, n, y, work, work_len, stream):
    _check(_lib().girih_mlp_forward(_vp(params), n_in, n_hidden, n_layers, _vp(x), n, _vp(y), _vp(work),
                                    int(work_len), _vp(stream)), "girih_mlp_forward")


def girih_mlp_loss_grad(params, n_in, n_hidden, n_layers, x, target, n, loss, grad, work, work_len, stream):
    _check(_lib().girih_mlp_loss_grad(_vp(params), n_in, n_hidden, n_layers, _vp(x), _vp(target), n, _vp(loss),
                                      _vp(grad), _vp(work), int(work_len), _vp(stream)), "girih_mlp_loss_grad")


def girih_mlp_adam(params, grad, m, v, count, lr, beta1, beta2, eps, step, stream):
    _check(_lib().girih_mlp_adam(_vp(params), _vp(grad), _vp(m), _vp(v), int(count), float(lr), float(beta1),
                                 float(beta2), float(eps), int(step), _vp(stream)), "girih_mlp_adam")
