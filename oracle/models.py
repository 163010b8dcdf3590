"""The paper's analytic models, written out plainly — TEST INFRASTRUCTURE ONLY.

The product's planner and tuner evaluate the same formulas in C++; these plain
versions exist to check them and to check the paper's own worked examples.

* ``cache_block_bytes``: Section "Cache block size model", equations for R = 1
  and for R > 1 — bytes of the wavefront cache block of one extruded diamond
  per byte of the leading dimension N_xb (multiply by N_xb for bytes).
* ``code_balance``: Section "Memory traffic model", equations for R = 1 and for
  R > 1 — main-memory bytes per lattice update of the blocked sweep in double
  precision, assuming the wavefront fits in cache.
* ``spatial_blocking_balance``: the non-temporal baseline quoted in the Results
  section (write-allocate counted unless non-temporal stores are used).
* ``flops_per_lup``: the paper's operation counts per lattice update (Results
  section) and the counts of the listings as written (used for the VALU bound).
"""


def cache_block_bytes(Dw, NF, R, ND):
    """C_S / N_xb of the single-thread wavefront diamond (paper's C_S model)."""
    if R == 1:
        Ww = Dw + NF - 2
        return ND * (Dw * Dw / 2 + Dw * (NF - 1)) + 2 * (Dw + Ww)
    Ww = Dw - 2 * R + NF
    return ND * Dw * (Dw / 2 - R + NF) + 2 * R * (Dw + Ww)


def code_balance(Dw, R, ND, word_bytes=8):
    """Blocked-sweep bytes per lattice update (paper's B_C; 16 = 2 x 8-byte words)."""
    per_diamond = (2 * Dw - 2 * R) + (ND * Dw + 2 * R)
    return 2 * word_bytes * R * per_diamond / (Dw * Dw)


def diamond_volume_per_plane(Dw, R):
    """Lattice updates of one extruded diamond per z-plane: Dw^2 / (2R)."""
    return Dw * Dw / (2 * R)


def spatial_blocking_balance(stencil_paper_form, nontemporal=False, word_bytes=8):
    """Bytes/LUP of the paper's spatially blocked baseline.

    7c/7v/25v: Jacobi form, reads V and the coefficient streams, writes U with
    write-allocate (one extra read of U) unless stores are non-temporal.
    25c (paper form): second order in time; U is read anyway, so no extra
    write-allocate transfer; the per-point array C is one more read stream.
    """
    if stencil_paper_form == "25c-leapfrog":
        return word_bytes * (3 + 1)
    n_coef = {"7c": 0, "7v": 7, "25v": 13}[stencil_paper_form]
    return word_bytes * (1 + n_coef + 1 + (0 if nontemporal else 1))


def flops_per_lup(stencil, as_written=True):
    """Floating-point operations per update.

    ``as_written``: count of the evaluation order of Listings 1-4 (first-order
    Jacobi form for 25c), which is what the GPU kernels execute.  Otherwise the
    paper's own counts for its forms (25c there is second order in time).
    """
    if as_written:
        return {"7c": 10, "7v": 13, "25c": 29, "25v": 37}[stencil]
    return {"7c": 7, "7v": 13, "25c-leapfrog": 33, "25v": 37}[stencil]
