"""ctypes wrapper around the C reference sweep — TEST INFRASTRUCTURE ONLY.

The reference result of the whole method is the naive two-buffer Jacobi sweep
(paper, Section "Background / Cache blocking"; captions of Listings 1-4):
temporal blocking only reorders independent point updates, so the blocked
schedule must end at exactly this result.  ``sweep`` runs it on host numpy
arrays in the layout ``(nz+2h, ny+2h, nx+2h)``; the work is done in
``oracle.c`` (built with ``gcc -O2 -ffp-contract=off``, OpenMP over z).

Parity status: pinned by ``tests/test_oracle_pins.py`` (sine eigenmode,
constant-field invariant, exact-rational brute force on 8^3, reflection,
light cone, linearity / time split, variable-vs-constant special case).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

STENCILS = {"7c": 0, "7v": 1, "25c": 2, "25v": 3, "25l": 4, "27b": 5}
RADIUS = {"7c": 1, "7v": 1, "25c": 4, "25v": 4, "25l": 4, "27b": 1}
N_COEF_ARRAYS = {"7c": 0, "7v": 7, "25c": 0, "25v": 13, "25l": 1, "27b": 0}
N_CONST_COEFS = {"7c": 2, "7v": 0, "25c": 5, "25v": 0, "25l": 5, "27b": 4}

_lib = None


def build(force=True):
    """Compile ``oracle.c`` into ``liboracle.so`` (plain gcc, no contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-fopenmp", _SRC, "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        for name, real in (("oracle_sweep_f64", ctypes.c_double), ("oracle_sweep_f32", ctypes.c_float)):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.c_int] + [ctypes.c_int64] * 6 + [
                ctypes.POINTER(real), ctypes.POINTER(real), ctypes.POINTER(real),
                ctypes.POINTER(ctypes.POINTER(real)), ctypes.c_int64]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def num_threads():
    return _load().oracle_num_threads()


def set_num_threads(n):
    _load().oracle_set_num_threads(int(n))


def sweep(stencil, buf0, buf1, T, const_coefs=None, coef_arrays=None):
    """Run T naive steps in place; return the index (T % 2) of the result buffer.

    ``buf0``/``buf1``: C-contiguous float64 or float32 arrays of shape
    ``(nz+2h, ny+2h, nx+2h)`` (no padding; h is the stencil radius).  ``buf0`` holds u^0 with
    its halo; ``buf1`` must carry the same halo (for the second-order-in-time
    ``25l`` its interior is u^{-1}).  ``const_coefs``: c0,c1 (7c), c0..c4
    (25c, 25l) or c0..c3 (27b).  ``coef_arrays``: 7 (7v), 13 (25v) or 1 (25l) arrays in the
    same layout as the field.
    """
    lib = _load()
    if stencil not in STENCILS:
        raise ValueError("unknown stencil %r" % (stencil,))
    dt = buf0.dtype
    if dt not in (np.float64, np.float32) or buf1.dtype != dt or buf0.shape != buf1.shape:
        raise ValueError("buffers must share a float64/float32 dtype and shape")
    for b in (buf0, buf1):
        if not b.flags["C_CONTIGUOUS"]:
            raise ValueError("buffers must be C-contiguous")
    real = ctypes.c_double if dt == np.float64 else ctypes.c_float
    fn = lib.oracle_sweep_f64 if dt == np.float64 else lib.oracle_sweep_f32
    h = RADIUS[stencil]
    nzp, nyp, pitch_x = buf0.shape
    nz, ny, nx = nzp - 2 * h, nyp - 2 * h, pitch_x - 2 * h
    ptr = lambda a: a.ctypes.data_as(ctypes.POINTER(real))
    keep = []
    c_ptr = ctypes.POINTER(real)()
    if N_CONST_COEFS[stencil]:
        c = np.ascontiguousarray(np.asarray(const_coefs, dtype=dt))
        if c.shape != (N_CONST_COEFS[stencil],):
            raise ValueError("stencil %s needs %d constant coefficients" % (stencil, N_CONST_COEFS[stencil]))
        keep.append(c)
        c_ptr = ptr(c)
    arr_ptr = ctypes.POINTER(ctypes.POINTER(real))()
    if N_COEF_ARRAYS[stencil]:
        if coef_arrays is None or len(coef_arrays) != N_COEF_ARRAYS[stencil]:
            raise ValueError("stencil %s needs %d coefficient arrays" % (stencil, N_COEF_ARRAYS[stencil]))
        arrs = []
        for a in coef_arrays:
            if a.dtype != dt or a.shape != buf0.shape or not a.flags["C_CONTIGUOUS"]:
                raise ValueError("coefficient arrays must match the field's dtype, shape and layout")
            arrs.append(a)
        keep.extend(arrs)
        table = (ctypes.POINTER(real) * len(arrs))(*[ptr(a) for a in arrs])
        keep.append(table)
        arr_ptr = ctypes.cast(table, ctypes.POINTER(ctypes.POINTER(real)))
    rc = fn(STENCILS[stencil], nx, ny, nz, h, pitch_x, nyp, ptr(buf0), ptr(buf1), c_ptr, arr_ptr, int(T))
    if rc != 0:
        raise ValueError("oracle rejected the arguments (rc=%d)" % rc)
    return int(T) % 2
