"""Host-side models of the diamond-row kernel's index logic (mwd_row_kernel).

These re-derive, in plain Python, the schedule rules the kernel applies per
workgroup and wave, and check them over many small configurations:

* stage coverage: every (level, row) a computed cell reads from the stage is
  provided exactly once (computed slots, input slots, stage duties of rows
  that compute nothing, out-of-span rows, halo rows), and nothing is staged
  outside the stage layout;
* address bounds: every coefficient load, halo load and prefetch load of the
  kernel's two loop bodies (ramp and steady) touches a plane inside the haloed
  array, and the steady range contains only steps whose level planes and
  stored planes lie inside the grid, for both loop unroll depths; the levels
  that rows computing nothing carry over are loaded one step before each
  plane of the grid is stored;
* x neighbours by lane moves (FP64, radius 1): with the kernel's edge-lane
  masks every lane inside the grid gets exactly the neighbours the stage
  holds, for zero and nonzero halos and every block of every x chunk;
* slot counts: the count the host uses to pick a kernel with fewer register
  slots per wave bounds what every wave of every diamond of the row holds,
  and the first and last rows of a run fit the H + 3 slots of the clipped-row
  kernel.

They need no GPU; the GPU parity tests check the kernel itself.
"""
import pytest


def partner(R, H, d):
    b, e = d // R, d % R
    b2 = H - 1 - b
    return b2 * R + e if b2 != b else b * R + (e ^ 1)


def stage_coverage_errors(R, DW, ny, T):
    H = DW // (2 * R); L = 2 * H
    w = lambda k: R * k if k < H else DW // 2 - R * (k - H)
    def row_levels(j, y, t_c):
        if j < 0 or j >= DW or y < 0 or y >= ny: return (1, 0)
        d = j - DW // 2 if j >= DW // 2 else DW // 2 - 1 - j
        b = d // R
        lo, hi = b + 1, L - 1 - b
        lo = max(lo, H - t_c); hi = min(hi, T - 1 + H - t_c)
        return (lo, hi) if lo <= hi else (1, 0)
    def in_layout(k, j):
        if k < 0 or k > L - 2: return False
        wk = w(k + 1)
        return DW // 2 - wk - R <= j < DW // 2 + wk + R
    n_rows = (T - 1) // H + 2
    errors = []
    for r in range(n_rows):
        t_c = r * H
        off = DW // 2 if r % 2 else 0
        nd = (ny + DW // 2 - off + DW - 1) // DW
        for m in range(nd):
            c = off + m * DW
            ybase = c - DW // 2
            kmax = min(L - 1, T - 1 + H - t_c)
            provided = {}
            def prov(k, j, who):
                if not in_layout(k, j):
                    errors.append(('out of layout', r, c, k, j, who)); return
                provided.setdefault((k, j), []).append(who)
            # waves
            waves = []
            for side in (0, 1):
                for d in range(DW // 2):
                    pd = partner(R, H, d)
                    if d < pd:
                        waves.append((side, d, pd))
            assert len(waves) == DW // 2, (R, DW)
            for side, dA, dB in waves:
                for d in (dA, dB):
                    j = DW // 2 + d if side == 0 else DW // 2 - 1 - d
                    y = ybase + j
                    kf, kl = row_levels(j, y, t_c)
                    for k in range(max(kf, 1), kl + 1):
                        if k <= L - 2: prov(k, j, 'comp')
                    # duties
                    if 0 <= y < ny:
                        ks = d // R + 1
                        kv = kf - 1 if kf <= kl else min(ks - 1, kmax - 1)
                        ok = lambda k: k >= 0 and t_c - H + k + 1 >= 0 and in_layout(k, j)
                        if kf <= kl: prov(kv, j, 'vring')
                        if kf > kl and ok(kv): prov(kv, j, 'pre1')
                        if ok(kv - 1): prov(kv - 1, j, 'pre2')
                    # out of span
                    if d // R == H - 1 and t_c < T:
                        jo = j + R if side == 0 else j - R
                        if -R <= ybase + jo < ny + R:
                            prov(H - 1, jo, 'preo')
            # halo rows
            for k in range(L - 1):
                for j in range(DW // 2 - w(k + 1) - R, DW // 2 + w(k + 1) + R):
                    y = ybase + j
                    if -R <= y < 0 or ny <= y < ny + R:
                        prov(k, j, 'halo')
            # needs
            for j in range(DW):
                y = ybase + j
                kf, kl = row_levels(j, y, t_c)
                for k in range(kf, kl + 1):
                    for jj in range(j - R, j + R + 1):
                        if (k - 1, jj) not in provided:
                            errors.append(('missing', r, c, k, j, jj))
            for key, who in provided.items():
                if len(who) > 1 and not set(who) <= {'halo', 'preo'}:
                    errors.append(('double', r, c, key, who))
    return errors



def bit_range(lo, hi):
    lo = max(lo, 0); hi = min(hi, 31)
    return 0 if lo > hi else (((2 << hi) - 1) & ~((1 << lo) - 1)) & 0xffffffff

def row_levels(R, DW, j, y, ny, t_c, T):
    H = DW // (2 * R); L = 2 * H
    if j < 0 or j >= DW or y < 0 or y >= ny: return (1, 0)
    d = j - DW // 2 if j >= DW // 2 else DW // 2 - 1 - j
    b = d // R
    lo, hi = max(b + 1, H - t_c), min(L - 1 - b, T - 1 + H - t_c)
    return (lo, hi) if lo <= hi else (1, 0)

def kernel_steps(R, DW, nz, NF=1, UNR=None, PD=1):
    """The wavefront steps of the kernel's three loops, as (zs, steady): zs
    counts slabs of NF planes, from -2*RZ in blocks of UNR; steps [zA, zB) run
    the steady body (mirrors mwd_tile)."""
    H = DW // (2 * R); L = 2 * H
    RZ = -(-R // NF); RING = 2 * RZ
    UNR = UNR or RING
    nzq = -(-nz // NF)
    nzs = nzq + RZ * L
    zA = -(-(RZ * L) // UNR) * UNR
    zB1 = nz // NF
    zB2 = (nz + R - NF) // NF - PD + 1
    zB0 = min(zB1, zB2)
    zB = max((zB0 // UNR) * UNR, zA)
    steps = []
    zb = -RING
    while zb < nzs:
        if zA <= zb < zB: break
        steps += [(zb + p, False) for p in range(UNR)]; zb += UNR
    while zb < zB:
        steps += [(zb + p, True) for p in range(UNR)]; zb += UNR
    while zb < nzs:
        steps += [(zb + p, False) for p in range(UNR)]; zb += UNR
    return [(zs, st) for zs, st in steps if st or zs < nzs], RZ, nzq


def load_bound_errors(R, DW, nx, ny, nz, T, ncoef, zh, fixed=True, NF=1, UNR=None):
    """Planes and rows of the coefficient and halo loads of both loop bodies,
    for every wave of every diamond of every row, lie inside the haloed arrays."""
    H = DW // (2 * R); L = 2 * H; NS = L + 2
    steps, RZ, nzq = kernel_steps(R, DW, nz, NF, UNR)
    bad = []
    def chk(kind, q, y, info):
        if not (-R <= q < nz + R) or not (-R <= y < ny + R):
            bad.append((kind, q, y) + info)
    waves = []
    for side in (0, 1):
        for d in range(DW // 2):
            pd = partner(R, H, d)
            if d < pd: waves.append((side, d, pd))
    n_rows = (T - 1) // H + 2
    for r in range(n_rows):
        t_c = r * H
        off = DW // 2 if r % 2 else 0
        nd = (ny + DW // 2 - off + DW - 1) // DW
        for m in range(nd):
            ybase = off + m * DW - DW // 2
            for side, dA, dB in waves:
                jA = DW // 2 + dA if side == 0 else DW // 2 - 1 - dA
                jB = DW // 2 + dB if side == 0 else DW // 2 - 1 - dB
                kfA, klA = row_levels(R, DW, jA, ybase + jA, ny, t_c, T)
                kfB, klB = row_levels(R, DW, jB, ybase + jB, ny, t_c, T)
                cmpA, cmpB = kfA <= klA, kfB <= klB
                sB = klA - kfA + 2 if cmpA else 1
                nB = klB - kfB + 2 if cmpB else 1
                baseA, baseB = kfA - 1, kfB - 1
                cm = 0; gos = {}
                for s in range(NS):
                    isB = s >= sB; t = s - sB if isB else s
                    valid = (cmpB and t < nB) if isB else cmpA
                    k = (baseB if isB else baseA) + t
                    j = jB if isB else jA
                    # (slabs above the window's first, row); unused slots: 0, row -R
                    gos[s] = (RZ * (L - k), ybase + j) if valid else (0, -R)
                    if valid and t >= 1: cm |= 1 << s
                maskA = bit_range(0, sB - 1)
                for zs, steady in steps:
                    for g in range(NF):
                        zS = 0xffffffff
                        if not steady:
                            pz = NF * zs + g
                            khz = pz // (NF * RZ) if pz >= 0 else -1
                            klz = (pz - nz) // (NF * RZ) + 1 if pz - nz >= 0 else 0
                            zS = (bit_range(klz - baseA, khz - baseA) & maskA) | (bit_range(klz - baseB + sB, khz - baseB + sB) & ~maskA & 0xffffffff)
                        for s in range(1, NS):
                            zv = (((cm & zS) if fixed else zS) >> s) & 1
                            dz, y = gos[s]
                            if ncoef and (steady or zv):
                                chk('coef', NF * (zs - RZ * L + dz) + g, y, (r, m, side, dA, zs, steady, s, g))
                            if not steady and not zv and not zh:
                                isB = s >= sB
                                k = baseB + (s - sB) if isB else baseA + s
                                q = NF * (zs - RZ * k) + g
                                if (((cm >> s) & 1) or not fixed) and -R <= q < nz + R:
                                    chk('halo', q, ybase + (jB if isB else jA), (r, m, zs, s, g))
    return bad



def check_prefetch(R, DW, ny, nz, T, PD=1, UNR=2, NF=1, steady_pd=None):
    """Planes of the prefetch loads (both bodies) stay inside [-R, nz+R); the
    steady range holds only steps whose level planes and stored planes lie
    inside the grid; every plane of the grid is stored once per level; the
    levels that rows computing nothing carry over (clipped-row kernel) are
    loaded for every plane of [0, nz) one step before the step that stores
    them.  UNR: steps per loop iteration (2, or 2*RZ where the kernel unrolls
    every ring phase); NF: planes per step (slabs).  steady_pd: the prefetch
    distance the steady range is computed for (default PD; another value
    models a wrong range)."""
    H = DW // (2 * R); L = 2 * H
    steps, RZ, nzq = kernel_steps(R, DW, nz, NF, UNR, PD if steady_pd is None else steady_pd)
    bad = []
    dzs = set(range(0, L)) | {H}
    for zs, steady in steps:
        if steady:
            for dz in dzs:
                for g in range(NF):
                    q = NF * (zs + PD - RZ * dz) + g
                    if not (-R <= q < nz + R):
                        bad.append((zs, dz, q))
            for k in range(L):
                for g in range(NF):
                    if not (0 <= NF * (zs - RZ * k) + g < nz) or not (0 <= NF * (zs - RZ * (k + 1)) + g < nz):
                        bad.append(('plane', zs, k, g))
    live = [zs for zs, steady in steps]
    if len(set(live)) != len(live) or live != sorted(live):
        bad.append(('step order', live[:5]))
    # stores: level k's stored slab at step zs is zs - RZ*(k+1); kept planes in [0, nz)
    for k in range(L):
        stored = [NF * (zs - RZ * (k + 1)) + g for zs in live for g in range(NF)]
        kept = sorted(q for q in stored if 0 <= q < nz)
        if kept != list(range(nz)):
            bad.append(('stores', k, kept[:4]))
    # carried levels: slab zs + PD loaded at step zs, stored at step zs + PD
    loaded = {NF * (zs + PD) + g for zs in live for g in range(NF) if 0 <= NF * (zs + PD) + g < nz}
    stored = {NF * zs + g for zs in live for g in range(NF) if 0 <= NF * zs + g < nz}
    if stored != set(range(nz)) or loaded != stored:
        bad.append(('carry', sorted(set(range(nz)) - stored)[:3], sorted(stored - loaded)[:3]))
    if steps and steps[0][0] % UNR != 0:
        bad.append(('phase', steps[0][0]))
    return bad




CONFIGS = [(1, (4, 8, 12, 16)), (4, (8, 16, 24))]


@pytest.mark.parametrize("R,DW", [(R, d) for R, ds in CONFIGS for d in ds])
def test_every_stage_read_is_provided_once(R, DW):
    for ny in list(range(1, 2 * DW + 5)) + [3 * DW + 1]:
        for T in range(1, 3 * DW // R + 3):
            e = stage_coverage_errors(R, DW, ny, T)
            assert not e, (R, DW, ny, T, e[:3])


NF_CONFIGS = [(1, 4, 2), (1, 8, 2), (1, 12, 2), (1, 16, 2), (4, 8, 2), (4, 16, 2), (4, 16, 4), (4, 8, 4), (1, 8, 3)]


@pytest.mark.parametrize("R,DW", [(R, d) for R, ds in CONFIGS for d in ds if d <= 16])
def test_loads_stay_inside_the_haloed_arrays(R, DW):
    for ny in (1, 3, 7, 2 * DW + 1):
        for nz in (1, 3, 9, 14):
            for T in (1, 3, 7):
                for zh in (True, False):
                    for unr in sorted({2, 2 * R}):
                        e = load_bound_errors(R, DW, 8, ny, nz, T, 1, zh, UNR=unr)
                        assert not e, (R, DW, ny, nz, T, zh, unr, e[:2])


@pytest.mark.parametrize("R,DW,NF", NF_CONFIGS)
def test_loads_stay_inside_the_haloed_arrays_with_wavefront_depth(R, DW, NF):
    RZ = -(-R // NF)
    for ny in (1, 3, 2 * DW + 1):
        for nz in (1, 2, 3, 5, 9, 14):
            for T in (1, 3, 7):
                for zh in (True, False):
                    for unr in sorted({2, 2 * RZ}):
                        e = load_bound_errors(R, DW, 8, ny, nz, T, 1, zh, NF=NF, UNR=unr)
                        assert not e, (R, DW, NF, ny, nz, T, zh, unr, e[:2])


def test_the_earlier_z_mask_is_caught():
    # the mask of an earlier build also covered unused slots: the model flags it
    assert load_bound_errors(1, 8, 129, 30, 14, 3, 7, True, fixed=False)
    assert not load_bound_errors(1, 8, 129, 30, 14, 3, 7, True, fixed=True)


@pytest.mark.parametrize("R,DW", [(R, d) for R, ds in CONFIGS for d in ds])
def test_prefetch_planes_and_steady_range(R, DW):
    for unr in sorted({2, 2 * R}):
        for nz in range(1, 40):
            e = check_prefetch(R, DW, 7, nz, 5, UNR=unr)
            assert not e, (R, DW, unr, nz, e[:3])


@pytest.mark.parametrize("R,DW,NF", NF_CONFIGS)
def test_prefetch_planes_and_steady_range_with_wavefront_depth(R, DW, NF):
    RZ = -(-R // NF)
    for unr in sorted({2, 2 * RZ}):
        for nz in range(1, 40):
            e = check_prefetch(R, DW, 7, nz, 5, UNR=unr, NF=NF)
            assert not e, (R, DW, NF, unr, nz, e[:3])


def test_a_steady_range_one_slab_too_long_is_caught():
    # a steady range that ignored the loads of the next slab (as for a zero
    # prefetch distance) would read past the haloed grid for NF = 2: the
    # model flags it
    assert any(check_prefetch(1, 8, 7, nz, 5, UNR=2, NF=2, steady_pd=0) for nz in range(2, 60))
    assert not any(check_prefetch(1, 8, 7, nz, 5, UNR=2, NF=2) for nz in range(2, 60))


def slots_needed(R, DW, t_c, T):
    """The host's slot count for a row (time clipping only, as the runtime)."""
    H = DW // (2 * R); L = 2 * H
    def slots(d):
        b = d // R
        lo, hi = max(b + 1, H - t_c), min(L - 1 - b, T - 1 + H - t_c)
        return hi - lo + 2 if lo <= hi else 1
    return max(slots(d) + slots(partner(R, H, d)) for d in range(DW // 2) if d < partner(R, H, d))


@pytest.mark.parametrize("R,DW", [(R, d) for R, ds in CONFIGS for d in ds])
def test_clipped_row_slot_counts(R, DW):
    H = DW // (2 * R); L = 2 * H
    waves = [(side, d, partner(R, H, d)) for side in (0, 1) for d in range(DW // 2) if d < partner(R, H, d)]
    for ny in (1, 5, 2 * DW + 3):
        for T in range(1, 4 * H + 4):
            n_rows = (T - 1) // H + 2
            for r in range(n_rows):
                t_c = r * H
                off = DW // 2 if r % 2 else 0
                nd = (ny + DW // 2 - off + DW - 1) // DW
                need = 0
                for m in range(nd):
                    ybase = off + m * DW - DW // 2
                    for side, dA, dB in waves:
                        jA = DW // 2 + dA if side == 0 else DW // 2 - 1 - dA
                        jB = DW // 2 + dB if side == 0 else DW // 2 - 1 - dB
                        kfA, klA = row_levels(R, DW, jA, ybase + jA, ny, t_c, T)
                        kfB, klB = row_levels(R, DW, jB, ybase + jB, ny, t_c, T)
                        nA = klA - kfA + 2 if kfA <= klA else 1
                        nB = klB - kfB + 2 if kfB <= klB else 1
                        need = max(need, nA + nB)
                bound = slots_needed(R, DW, t_c, T)
                assert need <= bound <= L + 2, (R, DW, ny, T, r, need, bound)
                if r == 0 or r == n_rows - 1:
                    assert bound <= H + 3, (R, DW, T, r, bound)


def xcd_tile(bx, by, gx, gy, nxcd=8):
    """The diamond-row kernel's renumbering of its workgroup (bx, by) of a
    gx x gy launch: XCD-contiguous runs of (diamond, x-chunk) tiles."""
    nb = gx * gy
    lid = bx + gx * by
    q, r = nb // nxcd, nb % nxcd
    x, pos = lid % nxcd, lid // nxcd
    t = (x * (q + 1) if x < r else r * (q + 1) + (x - r) * q) + pos
    return t % gx, t // gx


@pytest.mark.parametrize("nxcd", [1, 3, 8])
def test_workgroup_renumbering_is_a_bijection_with_contiguous_runs(nxcd):
    for gx in range(1, 9):
        for gy in range(1, 50):
            seen = {}
            for by in range(gy):
                for bx in range(gx):
                    seen[xcd_tile(bx, by, gx, gy, nxcd)] = (bx + gx * by) % nxcd
            assert sorted(seen) == sorted((c, d) for d in range(gy) for c in range(gx))
            # each XCD's tiles form one run in (diamond, chunk) order
            order = [seen[(c, d)] for d in range(gy) for c in range(gx)]
            runs = [order[0]] + [b for a, b in zip(order, order[1:]) if b != a]
            assert len(runs) == len(set(runs))


def dpp_neighbours(vals, stage_row, lane0_col, mask_rule):
    """x neighbours of the 64 lanes of one block as the FP64 radius-1 kernel
    forms them: lane i takes lane i-1's / i+1's register value (DPP wave
    shifts; a lane with no source gets 0), and lanes the mask names read both
    from the stage row instead."""
    n = len(vals)
    xm = [vals[i - 1] if i > 0 else 0.0 for i in range(n)]
    xp = [vals[i + 1] if i + 1 < n else 0.0 for i in range(n)]
    for i in range(n):
        if mask_rule(i, "m"):
            xm[i] = stage_row[lane0_col + i - 1]
        if mask_rule(i, "p"):
            xp[i] = stage_row[lane0_col + i + 1]
    return xm, xp


@pytest.mark.parametrize("nx", [1, 5, 63, 64, 65, 100, 130, 300])
def test_dpp_edge_masks_give_the_stage_values(nx):
    """For every block of every x chunk (zero and nonzero halo), lanes whose
    cell is inside the grid get exactly the x neighbours the stage holds:
    the DPP value where the neighbour lane staged its own register value,
    the stage otherwise (block ends, halo lanes' columns).  Only the
    columns 1 .. XL - 2 need them: from level 1 on the row's outermost
    columns lie outside the valid span [kR, XL - kR) of level k, and the
    stored columns [HX, XL - HX) lie inside it at every level up to L - 1.
    (The kernel masks the outermost lanes too; leaving them unmasked
    measured no faster.)"""
    import random
    R, XL, L = 1, 128, 12
    HX = R * (L - 1)
    x_own = XL - 2 * HX
    for k in range(1, L):
        assert k * R <= HX and XL - HX <= XL - k * R
    rnd = random.Random(nx)
    for zero_halo in (True, False):
        n_chunks = (nx + x_own - 1) // x_own
        for chunk in range(n_chunks):
            x0 = chunk * x_own - HX
            # a stage row: guard columns, then the XL cells; lanes stage their
            # register value, halo lanes the halo value (zero, or the loaded one)
            regs = [rnd.random() for _ in range(XL)]
            halo = {x: (0.0 if zero_halo else rnd.random()) for x in (-1, nx)}
            in_halo = lambda x: x in halo
            stage = [rnd.random()] * R + [halo[x0 + c] if in_halo(x0 + c) else regs[c] for c in range(XL)] + \
                [rnd.random()] * R
            for blk in range(XL // 64):
                cb = 64 * blk
                vals = regs[cb:cb + 64]

                def rule(i, side):
                    x = x0 + cb + i
                    return (i == 0 or in_halo(x - 1)) if side == "m" else (i == 63 or in_halo(x + 1))

                xm, xp = dpp_neighbours(vals, stage, R + cb, rule)
                for i in range(64):
                    x = x0 + cb + i
                    if 0 <= x < nx and 0 < cb + i < XL - 1:
                        assert xm[i] == stage[R + cb + i - 1], (nx, chunk, blk, i)
                        assert xp[i] == stage[R + cb + i + 1], (nx, chunk, blk, i)


def test_dpp_edge_masks_without_halo_lanes_fail():
    # a mask that forgets the halo-adjacent lanes hands lane x = 0 the halo
    # lane's register instead of the halo value: the check sees it
    R, XL, nx = 1, 128, 100
    regs = [float(c + 1) for c in range(XL)]
    x0 = -11
    stage = [9.0] + [0.0 if x0 + c in (-1, nx) else regs[c] for c in range(XL)] + [9.0]
    xm, _ = dpp_neighbours(regs[:64], stage, R, lambda i, side: i == 0 if side == "m" else i == 63)
    i = -x0          # lane of x = 0
    assert xm[i] != stage[R + i - 1]


def test_dpp_edge_masks_without_inner_block_ends_fail():
    # dropping the mask at the end of a 64-lane block inside the row (lane 63
    # of the first block, whose x + 1 neighbour sits in the next block's lane
    # 0) hands that lane the DPP fill value instead of the stage value
    R, XL = 1, 128
    regs = [float(c + 1) for c in range(XL)]
    stage = [9.0] + regs + [9.0]
    _, xp = dpp_neighbours(regs[:64], stage, R, lambda i, side: False)
    assert xp[63] != stage[R + 64]
