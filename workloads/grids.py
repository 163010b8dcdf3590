"""Workload definitions and seeded input generation.

Inputs follow the paper's experimental setup: cubic (or box) grids larger than
any cache, a domain-sized solution field, and for the variable-coefficient
stencils one domain-sized array per coefficient (Listings 2 and 4; Section
"Cache block size model" counts them as the N_D domain-sized streams).  The
paper does not give its initial data; the recipe used here is:

* generator ``numpy.random.Generator(PCG64(seed))``, ``.random()`` (U[0,1)),
  drawn in C order over the interior only, in this sequence: the field first,
  then the constant coefficients c0..c4 (25-point constant) or the coefficient
  arrays in index order (C0..C6, C00..C12);
* Dirichlet halo of width R (the stencil radius) fixed at zero in the field;
  coefficient halos are zero and never read;
* "normalised" coefficients are scaled so that the weights *as applied to a
  constant field* sum to one: c0 + 6*(c1+..+c4) for the 25-point constant
  stencil, C0+..+C6 per point for the 7-point variable stencil,
  C00 + 2*(C01+..+C12) per point for the 25-point variable stencil.  The sum
  is formed in float64, left to right, and each coefficient divided by it;
* single-precision inputs are the float64 values rounded to nearest;
* the second-order-in-time 25-point stencil (Listing 3 as printed, "25l")
  takes the field, then one per-point array C = 0.1 * U[0,1) (a squared
  Courant number, small enough for the scheme to stay stable), and fixed
  constants: the eighth-order central second-difference weights
  c1..c4 = 8/5, -1/5, 8/315, -1/560 and c0 = -6*(c1+c2+c3+c4), so that the
  bracket is a discrete Laplacian; both buffers start as u^0 (zero initial
  velocity);
* the 27-point box stencil ("27b", constant weights by distance class:
  centre, 6 faces, 12 edges, 8 corners) takes the field, then c0..c3 drawn
  and normalised so that c0 + 6*c1 + 12*c2 + 8*c3 = 1.
"""
import math
from dataclasses import dataclass, field as dc_field

import numpy as np

STENCILS = ("7c", "7v", "25c", "25v", "25l", "27b")
RADIUS = {"7c": 1, "7v": 1, "25c": 4, "25v": 4, "25l": 4, "27b": 1}
N_COEF_ARRAYS = {"7c": 0, "7v": 7, "25c": 0, "25v": 13, "25l": 1, "27b": 0}
N_CONST_COEFS = {"7c": 2, "7v": 0, "25c": 5, "25v": 0, "25l": 5, "27b": 4}


def laplacian8_weights():
    """c0..c4 of the eighth-order 3-D Laplacian used by the 25l workload."""
    c = [8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0]
    return np.array([-6.0 * math.fsum(c)] + c, dtype=np.float64)


@dataclass(frozen=True)
class Workload:
    name: str
    stencil: str
    nx: int
    ny: int
    nz: int
    T: int
    const_coefs: tuple = None      # fixed c0, c1 (7-point constant); None = drawn
    dtypes: tuple = ("f64",)
    note: str = ""

    @property
    def radius(self):
        return RADIUS[self.stencil]

    @property
    def lups(self):
        return self.nx * self.ny * self.nz * self.T


# The workloads of this study: the five of its configurations, the
# second-order 25-point stencil and the 27-point box stencil.  Sizes are interior points (x fastest).
WORKLOADS = {
    "7pt-const-64": Workload("7pt-const-64", "7c", 64, 64, 64, 16, (0.4, 0.1),
                             note="naive GPU sweep vs oracle; fits in cache"),
    "7pt-const-512": Workload("7pt-const-512", "7c", 512, 512, 512, 64, (0.4, 0.1), ("f64", "f32"),
                              note="blocked vs naive, bit-exact; headline throughput"),
    "25pt-const-512": Workload("25pt-const-512", "25c", 512, 512, 512, 32, None, ("f64", "f32"),
                               note="radius-4 star, c0..c4 drawn and normalised"),
    "25pt-var-384": Workload("25pt-var-384", "25v", 384, 384, 384, 32, None, ("f64", "f32"),
                             note="13 per-point coefficient arrays normalised per point"),
    "7pt-var-256x512x1024": Workload("7pt-var-256x512x1024", "7v", 256, 512, 1024, 64, None, ("f64", "f32"),
                                     note="7 per-point coefficient arrays; unseen by the tuner's training"),
    "25pt-leapfrog-512": Workload("25pt-leapfrog-512", "25l", 512, 512, 512, 32, None, ("f64", "f32"),
                                  note="Listing 3 as printed: second order in time, one per-point array"),
    "27pt-box-512": Workload("27pt-box-512", "27b", 512, 512, 512, 32, None, ("f64", "f32"),
                             note="27-point box, c0..c3 by distance class, drawn and normalised"),
}


def padded_shape(nx, ny, nz, h, pitch_x=None, pitch_y=None):
    """Shape (nz+2h, pitch_y, pitch_x) of a padded grid; pitches default to n+2h."""
    px = nx + 2 * h if pitch_x is None else int(pitch_x)
    py = ny + 2 * h if pitch_y is None else int(pitch_y)
    if px < nx + 2 * h or py < ny + 2 * h:
        raise ValueError("pitch smaller than the haloed extent")
    return (nz + 2 * h, py, px)


def to_padded(a, h, pitch_x=None, pitch_y=None, fill=0.0):
    """Copy an unpadded (nz+2h, ny+2h, nx+2h) array into a padded layout."""
    nzp, nyp, nxp = a.shape
    shape = padded_shape(nxp - 2 * h, nyp - 2 * h, nzp - 2 * h, h, pitch_x, pitch_y)
    out = np.full(shape, fill, dtype=a.dtype)
    out[:, :nyp, :nxp] = a
    return out


def from_padded(a, nx, ny, nz, h):
    """Unpadded (nz+2h, ny+2h, nx+2h) view of a padded array."""
    return a[:, : ny + 2 * h, : nx + 2 * h]


def _interior(n_shape, h, values, dtype=np.float64):
    nz, ny, nx = n_shape
    out = np.zeros((nz + 2 * h, ny + 2 * h, nx + 2 * h), dtype=dtype)
    out[h:h + nz, h:h + ny, h:h + nx] = values
    return out


def field_and_coefs(stencil, nx, ny, nz, seed=0, const_coefs=None, dtype="f64"):
    """Draw the initial field and the coefficients of one workload.

    Returns ``(u0, consts, arrays)``: ``u0`` of shape (nz+2h, ny+2h, nx+2h)
    with zero halo; ``consts`` a float64/float32 vector (c0,c1 or c0..c4) or
    None; ``arrays`` a list of coefficient arrays (same layout) or None.
    """
    if stencil not in STENCILS:
        raise ValueError("unknown stencil %r" % (stencil,))
    h = RADIUS[stencil]
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (nz, ny, nx)
    u0 = _interior(shape, h, rng.random(shape))
    consts = None
    arrays = None
    if stencil == "7c":
        consts = np.array(const_coefs if const_coefs is not None else (0.4, 0.1), dtype=np.float64)
    elif stencil == "25c":
        if const_coefs is not None:
            consts = np.array(const_coefs, dtype=np.float64)
        else:
            c = rng.random(5)
            s = math.fsum([c[0]] + [c[r] for r in range(1, 5) for _ in range(6)])
            consts = c / s
    elif stencil == "27b":
        if const_coefs is not None:
            consts = np.array(const_coefs, dtype=np.float64)
        else:
            c = rng.random(4)
            s = math.fsum([c[0]] + [c[1]] * 6 + [c[2]] * 12 + [c[3]] * 8)
            consts = c / s
    elif stencil == "25l":
        consts = laplacian8_weights() if const_coefs is None else np.array(const_coefs, dtype=np.float64)
        arrays = [_interior(shape, h, 0.1 * rng.random(shape))]
    elif stencil == "7v":
        raw = [rng.random(shape) for _ in range(7)]
        s = raw[0].copy()
        for a in raw[1:]:
            s += a
        arrays = [_interior(shape, h, a / s) for a in raw]
    else:  # 25v
        raw = [rng.random(shape) for _ in range(13)]
        s = raw[0].copy()
        for a in raw[1:]:
            s += 2.0 * a
        arrays = [_interior(shape, h, a / s) for a in raw]
    if dtype == "f32":
        u0 = u0.astype(np.float32)
        consts = None if consts is None else consts.astype(np.float32)
        arrays = None if arrays is None else [a.astype(np.float32) for a in arrays]
    elif dtype != "f64":
        raise ValueError("dtype must be 'f64' or 'f32'")
    return u0, consts, arrays
