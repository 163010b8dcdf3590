"""CPU model of the dependency-driven schedule's waits (mwd_sweep_kernel):
every earlier tile that a tile conflicts with -- it reads cells the other
wrote, or writes cells the other read or wrote, in the same array -- is
among the tiles the tile waits for, directly or through the tiles those
wait for.  Exact cell sets on small grids; the wait set is the kernel's
(two diamonds of the previous row, x chunks within kx) with kx as the host
computes it."""
import itertools

import pytest


def tiles(R, DW, ny, nx, xo, n_rows):
    nch = -(-nx // xo)
    out = []
    for r in range(n_rows):
        off = DW // 2 if r % 2 else 0
        nd = (ny + DW // 2 - off + DW - 1) // DW
        for m in range(nd):
            for c in range(nch):
                out.append((r, m, c))
    return out, nch


def cells(R, DW, ny, nx, xo, XL, tile):
    """(rows read, cols read, rows written, cols written) of a tile, in the interior."""
    r, m, c = tile
    L = DW // R
    HX = R * (L - 1)
    yc = (DW // 2 if r % 2 else 0) + m * DW
    x0 = c * xo - HX
    rows_r = set(range(max(0, yc - DW // 2 - R), min(ny, yc + DW // 2 + R)))
    cols_r = set(range(max(0, x0 - R), min(nx, x0 + XL + R)))
    rows_w = set(range(max(0, yc - DW // 2), min(ny, yc + DW // 2)))
    cols_w = set(range(c * xo, min(nx, (c + 1) * xo)))
    return rows_r, cols_r, rows_w, cols_w


def kernel_waits(R, DW, ny, nx, xo, XL, tile, nch):
    r, m, c = tile
    if r == 0:
        return set()
    L = DW // R
    HX = R * (L - 1)
    kx = max(1, -(-(XL - HX + R) // xo) - 1)
    off_prev = DW // 2 if (r - 1) % 2 else 0
    nd_prev = (ny + DW // 2 - off_prev + DW - 1) // DW
    m_lo = m if r % 2 else m - 1
    return {(r - 1, mm, cc) for mm in (m_lo, m_lo + 1) for cc in range(c - kx, c + kx + 1)
            if 0 <= mm < nd_prev and 0 <= cc < nch}


def conflicts(R, DW, ny, nx, xo, XL, a, b):
    """Tile a (later row) and b (earlier row) touch a common cell of one array
    with at least one of them writing it.  Even rows read array 0 and write
    array 1, odd rows the reverse."""
    ra, ca, wa, cwa = cells(R, DW, ny, nx, xo, XL, a)
    rb, cb, wb, cwb = cells(R, DW, ny, nx, xo, XL, b)
    read_a, write_a = a[0] % 2, 1 - a[0] % 2
    read_b, write_b = b[0] % 2, 1 - b[0] % 2
    def meet(r1, c1, r2, c2):
        return bool(r1 & r2) and bool(c1 & c2)
    return ((read_a == write_b and meet(ra, ca, wb, cwb)) or (write_a == read_b and meet(wa, cwa, rb, cb))
            or (write_a == write_b and meet(wa, cwa, wb, cwb)))


def missing_waits(R, DW, ny, nx, xo, XL, n_rows, waits=kernel_waits):
    ts, nch = tiles(R, DW, ny, nx, xo, n_rows)
    direct = {t: waits(R, DW, ny, nx, xo, XL, t, nch) for t in ts}
    closure = {}
    for t in ts:   # rows in order: the closure of earlier tiles is known
        cl = set()
        for d in direct[t]:
            cl |= {d} | closure[d]
        closure[t] = cl
    bad = []
    for a in ts:
        for b in ts:
            if b[0] < a[0] and b not in closure[a] and conflicts(R, DW, ny, nx, xo, XL, a, b):
                bad.append((a, b))
    return bad


@pytest.mark.parametrize("R,DW,XL,xo", [(1, 8, 128, 114), (1, 8, 128, 40), (1, 12, 128, 103), (1, 12, 128, 86),
                                        (1, 12, 128, 30), (1, 16, 64, 34), (4, 8, 64, 56), (4, 8, 128, 60),
                                        (4, 16, 64, 40), (4, 16, 64, 24), (4, 16, 128, 104)])
def test_every_conflicting_tile_is_waited_for(R, DW, XL, xo):
    for ny in (DW // 2 + 1, 2 * DW + 3):
        for nx in (xo, 3 * xo - 1):
            e = missing_waits(R, DW, ny, nx, xo, XL, 5)
            assert not e, (R, DW, XL, xo, ny, nx, e[:3])


def test_a_narrower_wait_is_caught():
    # waiting only on the tile's own chunk misses the x-halo neighbours
    def own_chunk_only(R, DW, ny, nx, xo, XL, tile, nch):
        return {t for t in kernel_waits(R, DW, ny, nx, xo, XL, tile, nch) if t[2] == tile[2]}
    assert missing_waits(1, 12, 27, 300, 103, 128, 4, own_chunk_only)
    # and waiting on one diamond misses the other half of the tile's rows
    def one_diamond(R, DW, ny, nx, xo, XL, tile, nch):
        r, m, c = tile
        return {t for t in kernel_waits(R, DW, ny, nx, xo, XL, tile, nch) if t[1] == (m if r % 2 else m - 1)}
    assert missing_waits(1, 12, 27, 300, 103, 128, 4, one_diamond)
