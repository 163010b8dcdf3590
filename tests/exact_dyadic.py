"""Exact (rational) evaluation of the stencil sweeps on tiny grids.

Every float64 value is a dyadic rational N / 2^E.  A Jacobi step is a linear
map with dyadic weights, so the exact state after any number of steps is again
dyadic: we keep integer numerators (numpy object arrays of Python ints) and one
exponent per state.  The stencils are written here as term tables — a
coefficient index and the list of neighbour offsets it multiplies — taken from
Listings 1-4 (first-order Jacobi form of Listing 3's bracket), independently of
the C oracle's loop code.
"""
from fractions import Fraction

import numpy as np

# (coefficient index, [(dz, dy, dx), ...]) — Listings 1-4.
def _axis(r):
    return [(0, 0, r), (0, 0, -r)], [(0, r, 0), (0, -r, 0)], [(r, 0, 0), (-r, 0, 0)]


def term_table(stencil):
    c = [(0, 0, 0)]
    if stencil == "7c":
        x, y, z = _axis(1)
        return [(0, c), (1, x), (1, y), (1, z)]
    if stencil == "7v":
        return [(0, c), (1, [(0, 0, 1)]), (2, [(0, 0, -1)]), (3, [(0, 1, 0)]), (4, [(0, -1, 0)]),
                (5, [(1, 0, 0)]), (6, [(-1, 0, 0)])]
    if stencil == "25c":
        t = [(0, c)]
        for r in range(1, 5):
            x, y, z = _axis(r)
            t.append((r, x + y + z))
        return t
    if stencil == "25v":
        t = [(0, c)]
        for r in range(1, 5):
            x, y, z = _axis(r)
            t += [(3 * r - 2, x), (3 * r - 1, y), (3 * r, z)]
        return t
    if stencil == "27b":
        # the 26 neighbours of the 3x3x3 box, weight by how many of the three
        # offsets are nonzero (faces 1, edges 2, corners 3)
        import itertools
        offs = [d for d in itertools.product((-1, 0, 1), repeat=3) if d != (0, 0, 0)]
        return [(0, c)] + [(m, [d for d in offs if sum(1 for a in d if a) == m]) for m in (1, 2, 3)]
    raise ValueError(stencil)


def _to_dyadic(values):
    """Common-exponent integer numerators of an array of finite floats."""
    flat = [Fraction(float(v)) for v in np.asarray(values, dtype=np.float64).ravel()]
    E = 0
    for f in flat:
        d = f.denominator
        E = max(E, d.bit_length() - 1)
    nums = np.empty(len(flat), dtype=object)
    for n, f in enumerate(flat):
        nums[n] = f.numerator * ((1 << E) // f.denominator)
    return nums.reshape(np.shape(values)), E


def exact_sweep(stencil, u0, T, consts=None, arrays=None):
    """Exact state after T steps, as a numpy object array of Fractions.

    ``u0`` is (nz+2h, ny+2h, nx+2h) float64 with its fixed halo; ``consts`` or
    ``arrays`` as for the oracle.
    """
    h = 1 if stencil in ("7c", "7v", "27b") else 4
    table = term_table(stencil)
    N, E = _to_dyadic(u0)
    if arrays is not None:
        A, ec = _to_dyadic(np.stack([np.asarray(a, dtype=np.float64) for a in arrays]))
        coef = [A[m] for m in range(A.shape[0])]
    else:
        A, ec = _to_dyadic(np.asarray(consts, dtype=np.float64))
        coef = [A[m] for m in range(A.shape[0])]
    nzp, nyp, nxp = u0.shape
    nz, ny, nx = nzp - 2 * h, nyp - 2 * h, nxp - 2 * h
    inner = (slice(h, h + nz), slice(h, h + ny), slice(h, h + nx))
    scale = 1 << ec
    for _ in range(T):
        new = N * scale                       # halo: same value, new exponent
        acc = None
        for m, offs in table:
            s = None
            for dz, dy, dx in offs:
                v = N[h + dz:h + dz + nz, h + dy:h + dy + ny, h + dx:h + dx + nx]
                s = v if s is None else s + v
            cm = coef[m][inner] if arrays is not None else coef[m]
            term = cm * s
            acc = term if acc is None else acc + term
        new[inner] = acc
        N, E = new, E + ec
    den = 1 << E
    out = np.empty(N.shape, dtype=object)
    for idx in np.ndindex(N.shape):
        out[idx] = Fraction(N[idx], den)
    return out


def to_float(exact):
    return np.vectorize(float, otypes=[np.float64])(exact)
