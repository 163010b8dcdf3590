"""Relaxed synchronisation within a diamond tile (paper, Section "Multi-core
wavefront temporal blocking": a thread waits only for the threads whose data
it uses): the kernel replaces the workgroup barriers of a wavefront step by
waits on the step counters of a fixed set of waves.  This test derives, from
the tile's geometry alone, which waves must wait for which, and checks the
set the kernel computes (printed by a host build of its header) against it.

The LDS traffic between waves of a tile: level k+1 of row j reads level k of
the rows within R of j (x and y neighbours; z neighbours stay in registers);
each wave stages the levels of its own two rows, and for a row of the
outermost block of R rows also the row R beyond it (outside the diamond);
a row's x range is split among the waves of its row pair (the x slices),
which read each other's edge cells.  So wave w must wait for wave v when w
reads a row v stages (before updating), or v reads a row w stages (before
staging over it), or both belong to the same row pair."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def kernel_masks(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("wn") / "wave_neighbours")
    src = os.path.join(ROOT, "tests", "native", "wave_neighbours.cpp")
    cmd = ["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_1510_04995_amd", "csrc"), src,
           "-o", exe]
    if not os.path.exists(cmd[0]):
        pytest.skip("hipcc not available")
    subprocess.run(cmd, check=True, capture_output=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    masks = {}
    for line in out.split("\n"):
        if line.strip():
            v = [int(x) for x in line.split()]
            masks[tuple(v[:3])] = v[3:]
    return masks


def row_pairs(R, DW):
    """The two rows of each row pair: half-distance d from the centre (row
    DW/2 + d on the right, DW/2 - 1 - d on the left) pairs with the row of
    the mirrored block (block d // R with H - 1 - d // R, same offset in the
    block; a middle block pairs neighbouring offsets), so that the pair's two
    rows compute L levels together.  Pairs 0 .. DW/4-1: right half."""
    H = DW // (2 * R)

    def partner(d):
        b, e = divmod(d, R)
        b2 = H - 1 - b
        return b2 * R + e if b2 != b else b * R + (e ^ 1)
    halves = [(d, partner(d)) for d in range(DW // 2) if d < partner(d)]
    pairs = [(DW // 2 + a, DW // 2 + b) for a, b in halves] + [(DW // 2 - 1 - a, DW // 2 - 1 - b) for a, b in halves]
    # every row of the diamond belongs to exactly one pair, and the levels of
    # a pair's rows add up to L
    assert sorted(j for p in pairs for j in p) == list(range(DW))
    for a, b in halves:
        assert (2 * H - 1 - 2 * (a // R)) + (2 * H - 1 - 2 * (b // R)) == 2 * H
    return pairs


def needed(R, DW, WX):
    pairs = row_pairs(R, DW)
    npairs = len(pairs)
    owner = {j: q for q, p in enumerate(pairs) for j in p}
    # rows staged by each pair: its own, and the rows beyond the diamond
    # (staged by the owner of the row R further in)
    writes = {q: set(p) for q, p in enumerate(pairs)}
    for r in list(range(-R, 0)) + list(range(DW, DW + R)):
        writes[owner[r + R if r < 0 else r - R]].add(r)
    reads = {q: {j + o for j in p for o in range(-R, R + 1)} for q, p in enumerate(pairs)}
    nw = npairs * WX
    out = []
    for w in range(nw):
        m = 0
        for v in range(nw):
            if v == w:
                continue
            a, b = w % npairs, v % npairs
            if a == b or reads[a] & writes[b] or reads[b] & writes[a]:
                m |= 1 << v
        out.append(m)
    return out


SHAPES = [(1, DW, wx) for DW in (4, 8, 12, 16) for wx in (1, 2, 3, 4) if DW // 2 * wx <= 16] + \
         [(1, 24, 1), (1, 32, 1)] + [(4, DW, wx) for DW in (8, 16) for wx in (1, 2, 3, 4) if DW // 2 * wx <= 16] + \
         [(4, 24, 1), (4, 32, 1)]


@pytest.mark.parametrize("R,DW,WX", SHAPES)
def test_kernel_waits_on_exactly_the_waves_it_shares_rows_with(kernel_masks, R, DW, WX):
    got = kernel_masks[(R, DW, WX)]
    want = needed(R, DW, WX)
    assert got == want, (R, DW, WX, got, want)


def test_planted_mistakes_are_caught(kernel_masks):
    """Planted mistakes in the model -- a reach of R - 1 rows -- give sets
    that differ from the kernel's, so the comparison sees such a slip.  (The
    other x slices of a row pair, and the rows beyond the diamond, are
    covered twice over: slices share their rows, and a row beyond is read
    only by rows next to the one that stages it.)"""
    def model(R, DW, WX, reach, slices):
        pairs = row_pairs(R, DW)
        writes = {q: set(p) for q, p in enumerate(pairs)}
        reads = {q: {j + o for j in p for o in range(-reach, reach + 1)} for q, p in enumerate(pairs)}
        n = len(pairs)
        return [sum(1 << v for v in range(n * WX) if v != w and
                    ((slices and w % n == v % n) or reads[w % n] & writes[v % n] or reads[v % n] & writes[w % n]))
                for w in range(n * WX)]
    assert model(1, 12, 2, 1, True) == kernel_masks[(1, 12, 2)]
    assert model(1, 12, 2, 0, True) != kernel_masks[(1, 12, 2)]
    assert model(4, 16, 1, 3, True) != kernel_masks[(4, 16, 1)]
    assert model(1, 12, 2, 1, False) == kernel_masks[(1, 12, 2)]


def test_neighbour_sets_are_local_for_the_seven_point_tile(kernel_masks):
    """For the 7-point default tile (Dw = 12, two x slices per row pair) a
    wave waits for at most 5 of the 11 other waves: the waits stay local."""
    assert max(bin(m).count("1") for m in kernel_masks[(1, 12, 2)]) <= 5
