"""Host-side checks of libgirih.so that need no GPU: the library loads, exports
every function declared in include/girih.h, and validates plans on the host
(plan creation touches no device)."""
import ctypes
import os
import re

import pytest

from paper_1510_04995_amd import girih as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "girih.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(girih_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("girih_plan", "girih_run", "girih_tune", "girih_plan_info", "girih_destroy", "girih_strerror"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(G.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) <= set(G.SIGNATURES)


def test_strerror_and_version():
    assert G.girih_strerror(0) == "ok"
    assert "invalid" in G.girih_strerror(-1)
    assert "gfx950" in G.girih_version()


def grid(n=32, h=1, **kw):
    return G.make_grid(n, n, n, h, **kw)


def test_plan_defaults_and_info():
    p = G.girih_plan("7c", "f64", grid(), (0.4, 0.1), "mwd")
    params, lds, bpl = G.girih_plan_info(p)
    assert params["diamond_width"] % 4 == 0 and params["wavefront_depth"] == 1
    assert params["threads_y"] == params["diamond_width"] // 2
    assert 0 < lds <= 160 * 1024
    assert 0 < bpl < 16
    G.girih_destroy(p)
    p = G.girih_plan("7v", "f32", grid(), None, "naive")
    params, lds, bpl = G.girih_plan_info(p)
    assert bpl == pytest.approx(9 * 4)
    G.girih_destroy(p)


@pytest.mark.parametrize("bad", [
    dict(stencil="7c", g=lambda: grid(h=2), c=(0.4, 0.1)),            # halo != R
    dict(stencil="25c", g=lambda: grid(h=1), c=(1, 0, 0, 0, 0)),       # halo != R
    dict(stencil="7c", g=lambda: G.make_grid(0, 4, 4, 1), c=(0.4, 0.1)),  # empty
    dict(stencil="7c", g=lambda: grid(pitch_x=10), c=(0.4, 0.1)),     # pitch too small
    dict(stencil="7c", g=lambda: grid(), c=None),                     # missing constants
])
def test_plan_rejects_invalid(bad):
    with pytest.raises(G.GirihError) as e:
        G.girih_plan(bad["stencil"], "f64", bad["g"](), bad["c"], "mwd")
    assert e.value.code == G.E_INVALID


def test_plan_rejects_bad_tile_params():
    g = grid()
    with pytest.raises(G.GirihError) as e:
        G.girih_plan("7c", "f64", g, (0.4, 0.1), "mwd", {"diamond_width": 6})   # not a multiple of 4
    assert e.value.code == G.E_INVALID
    with pytest.raises(G.GirihError) as e:
        G.girih_plan("25c", "f64", G.make_grid(32, 32, 32, 4), (1, 0, 0, 0, 0), "mwd", {"diamond_width": 12})
    assert e.value.code == G.E_INVALID
    with pytest.raises(G.GirihError) as e:
        G.girih_plan("7c", "f64", g, (0.4, 0.1), "mwd", {"diamond_width": 8, "threads_x": 128, "tile_x": 4096})
    assert e.value.code == G.E_LDS
    with pytest.raises(G.GirihError) as e:
        G.girih_plan("7c", "f64", g, (0.4, 0.1), "mwd", {"diamond_width": 40})
    assert e.value.code == G.E_UNSUPPORTED
    with pytest.raises(G.GirihError) as e:
        G.girih_plan("7c", "f64", g, (0.4, 0.1), "mwd", {"wavefront_depth": 3})
    assert e.value.code == G.E_UNSUPPORTED
    with pytest.raises(G.GirihError) as e:
        G.girih_plan("7c", "f64", g, (0.4, 0.1), "naive", {"threads_x": 64, "threads_y": 8})  # 512 > 256
    assert e.value.code == G.E_INVALID


def test_mwd_variable_coefficient_shapes():
    """Blocked plans of the variable-coefficient and the second-order-in-time
    stencils exist for the registered (spill-free) shapes only."""
    for st, h, dt, dw in (("7v", 1, "f64", 8), ("7v", 1, "f32", 8), ("25v", 4, "f64", 8), ("25v", 4, "f32", 16)):
        p = G.girih_plan(st, dt, grid(h=h), None, "mwd")
        assert G.girih_plan_info(p)[0]["diamond_width"] == dw
        G.girih_destroy(p)
    with pytest.raises(G.GirihError) as e:
        G.girih_plan("7v", "f64", grid(), None, "mwd", {"diamond_width": 12})     # spills: not compiled
    assert e.value.code == G.E_UNSUPPORTED
    for dt in ("f64", "f32"):
        p = G.girih_plan("25l", dt, grid(h=4), (0.1, 0.1, 0.1, 0.1, 0.1), "mwd")
        assert G.girih_plan_info(p)[0]["diamond_width"] == 16
        G.girih_destroy(p)
    with pytest.raises(G.GirihError) as e:
        G.girih_plan("25l", "f64", grid(h=4), (0.1, 0.1, 0.1, 0.1, 0.1), "mwd", {"diamond_width": 24})
    assert e.value.code == G.E_UNSUPPORTED


def test_run_rejects_without_launch():
    p = G.girih_plan("7v", "f64", grid(), None, "naive")
    with pytest.raises(G.GirihError) as e:
        G.girih_run(p, 0, 0, [], 4, 0)                 # null buffers
    assert e.value.code == G.E_INVALID
    with pytest.raises(G.GirihError) as e:
        G.girih_run(p, 4096, 8192, [16] * 6, 4, 0)     # 6 coefficient arrays for 7v
    assert e.value.code == G.E_INVALID
    with pytest.raises(G.GirihError) as e:
        G.girih_run(p, 4096, 8192, [16] * 7, -1, 0)    # T < 0
    assert e.value.code == G.E_INVALID
    G.girih_destroy(p)


def test_candidates_cover_compiled_variants():
    p = G.girih_plan("7c", "f64", G.make_grid(512, 512, 512, 1), (0.4, 0.1), "mwd")
    c = G.girih_candidates(p)
    dws = {q["diamond_width"] for q in c}
    assert {4, 8, 12, 16} <= dws
    for q in c:
        assert q["threads_y"] == q["diamond_width"] // 2
        # a row spans threads_x * cells_per_lane cells: the owned tile plus R*(L-1) = Dw-R on each side
        assert 8 <= q["tile_x"] <= q["threads_x"] * q["cells_per_lane"] - 2 * (q["diamond_width"] - 1)
    G.girih_destroy(p)
    p = G.girih_plan("25c", "f32", G.make_grid(384, 384, 384, 4), (1, 0, 0, 0, 0), "mwd")
    c = G.girih_candidates(p)
    assert all(q["diamond_width"] % 8 == 0 for q in c) and c
    G.girih_destroy(p)


def test_box_plans():
    """The 27-point box stencil: a naive plan streams the field pair (16 B per
    update in FP64) with register columns by default (variant 1: 62 x cells
    per wave, in FP64 8 rows per lane and 64 x 2 threads), and the cached
    variant on request;
    blocks wider than 256 threads or rows per lane not compiled are refused.
    The blocked plan takes Dw = 8 in FP64 and 12 in FP32 (which also offers
    8), row launches only, with three-plane stage rows."""
    g = G.make_grid(64, 48, 40, 1)
    c = (0.2, 0.05, 0.02, 0.01)
    p = G.girih_plan("27b", "f64", g, c, "naive")
    q, lds, bytes_per_lup = G.girih_plan_info(p)
    assert bytes_per_lup == 16.0 and lds == 0
    assert (q["variant"], q["threads_x"], q["threads_y"], q["cells_per_lane"], q["tile_x"], q["tile_y"]) == \
        (1, 64, 2, 8, 62, 16)
    G.girih_destroy(p)
    for params, want in (({"variant": 0, "threads_x": 64, "threads_y": 4}, (0, 64, 4, 1)),
                         ({"variant": 1, "threads_x": 64, "threads_y": 2, "cells_per_lane": 8}, (62, 16, 2, 8)),
                         ({"variant": 1, "threads_x": 64, "threads_y": 4, "cells_per_lane": 2}, (62, 8, 4, 2))):
        p = G.girih_plan("27b", "f32", g, c, "naive", params)
        q, _, _ = G.girih_plan_info(p)
        if params["variant"] == 0:
            assert (q["variant"], q["threads_x"], q["threads_y"], q["cells_per_lane"]) == want
        else:
            assert (q["tile_x"], q["tile_y"], q["threads_y"], q["cells_per_lane"]) == want
        G.girih_destroy(p)
    for params in ({"variant": 1, "threads_x": 64, "threads_y": 8}, {"variant": 1, "threads_x": 64, "threads_y": 4,
                                                                     "cells_per_lane": 3}):
        with pytest.raises(G.GirihError) as e:
            G.girih_plan("27b", "f64", g, c, "naive", params)
        assert e.value.code == G.E_UNSUPPORTED
    for dt, dws, dflt in (("f64", {8}, 8), ("f32", {8, 12}, 12)):
        p = G.girih_plan("27b", dt, g, c, "mwd")
        q, lds, _ = G.girih_plan_info(p)
        assert (q["diamond_width"], q["wavefront_depth"], q["variant"]) == (dflt, 1, 0) and lds <= 160 * 1024
        cands = G.girih_candidates(p)
        assert {x["diamond_width"] for x in cands} == dws and {x["variant"] for x in cands} == {0}
        G.girih_destroy(p)
    for params in ({"variant": 1}, {"wavefront_depth": 2}, {"diamond_width": 16}):
        with pytest.raises(G.GirihError) as e:
            G.girih_plan("27b", "f64", g, c, "mwd", params)
        assert e.value.code == G.E_UNSUPPORTED
    with pytest.raises(G.GirihError) as e:
        G.girih_plan("27b", "f64", G.make_grid(64, 48, 40, 2), c, "naive")   # halo != R
    assert e.value.code == G.E_INVALID


def test_star_register_column_plans():
    """Naive variant 2 (register columns) for the constant-coefficient star
    stencils: tile_x = 64 - 2R cells stored per wave, tile_y = waves x rows
    per lane; refused for the stencils with coefficient arrays or two time
    levels, for blocks that are not 64 lanes wide, and for rows per lane not
    compiled."""
    for st, dt, r, w, ky in (("7c", "f64", 1, 4, 8), ("7c", "f32", 1, 2, 2), ("25c", "f32", 4, 2, 4),
                              ("25c", "f64", 4, 4, 2)):
        g = G.make_grid(100, 50, 30, r)
        c = (0.4, 0.1) if st == "7c" else (0.2, 0.05, 0.04, 0.03, 0.0133)
        p = G.girih_plan(st, dt, g, c, "naive", {"variant": 2, "threads_x": 64, "threads_y": w,
                                                  "cells_per_lane": ky, "tile_z": 9})
        q, lds, _ = G.girih_plan_info(p)
        assert (q["variant"], q["tile_x"], q["tile_y"], q["cells_per_lane"], q["tile_z"], lds) == \
            (2, 64 - 2 * r, w * ky, ky, 9, 0)
        G.girih_destroy(p)
    # the FP32 default naive plans of both stencils; FP64 keeps the plane tiles
    for st, dt, r, want in (("7c", "f32", 1, (2, 2, 4, 62, 12)), ("25c", "f32", 4, (2, 2, 8, 56, 12)),
                            ("7c", "f64", 1, (1, 16, 1, 64, 128)), ("25c", "f64", 4, (1, 16, 1, 64, 128))):
        c = (0.4, 0.1) if st == "7c" else (0.2, 0.05, 0.04, 0.03, 0.0133)
        p = G.girih_plan(st, dt, G.make_grid(512, 512, 512, r), c, "naive")
        q = G.girih_plan_info(p)[0]
        assert (q["variant"], q["threads_y"], q["cells_per_lane"], q["tile_x"], q["tile_z"]) == want, (st, dt, q)
        G.girih_destroy(p)
    g = G.make_grid(100, 50, 30, 1)
    for st, params, code in (("7v", {"variant": 2, "threads_x": 64, "threads_y": 4}, G.E_UNSUPPORTED),
                             ("7c", {"variant": 2, "threads_x": 128, "threads_y": 2}, G.E_INVALID),
                             ("7c", {"variant": 2, "threads_x": 64, "threads_y": 4, "cells_per_lane": 3},
                              G.E_UNSUPPORTED),
                             ("7c", {"variant": 3, "threads_x": 64, "threads_y": 4}, G.E_UNSUPPORTED)):
        c = (0.4, 0.1) if st == "7c" else None
        with pytest.raises(G.GirihError) as e:
            G.girih_plan(st, "f64", g, c, "naive", params)
        assert e.value.code == code, (st, params)
    g4 = G.make_grid(100, 50, 30, 4)
    for st in ("25v", "25l"):
        with pytest.raises(G.GirihError) as e:
            G.girih_plan(st, "f64", g4, None if st == "25v" else (0.2, 0.05, 0.04, 0.03, 0.0133), "naive",
                         {"variant": 2, "threads_x": 64, "threads_y": 4})
        assert e.value.code == G.E_UNSUPPORTED


def test_default_schedules():
    """The default plan takes the dependency-driven schedule (variant 1)
    where it measured faster -- 25-point constant and 7-point variable in
    FP64 -- and row launches elsewhere; a default shape asked for explicitly
    keeps the variant it is given."""
    cases = (("25c", "f64", 4, (0.2, 0.05, 0.04, 0.03, 0.0133), 1), ("7v", "f64", 1, None, 1),
             ("7c", "f64", 1, (0.4, 0.1), 0), ("25c", "f32", 4, (0.2, 0.05, 0.04, 0.03, 0.0133), 0),
             ("7v", "f32", 1, None, 0))
    for st, dt, h, c, var in cases:
        p = G.girih_plan(st, dt, G.make_grid(64, 64, 64, h), c, "mwd")
        assert G.girih_plan_info(p)[0]["variant"] == var, (st, dt)
        G.girih_destroy(p)
    p = G.girih_plan("25c", "f64", G.make_grid(64, 64, 64, 4), cases[0][3], "mwd", {"diamond_width": 16})
    assert G.girih_plan_info(p)[0]["variant"] == 0
    G.girih_destroy(p)


def test_lds_budget_prunes_candidates():
    """The user's on-chip budget (the paper's cache size) leaves out every
    candidate whose workgroup needs more LDS; 0 restores all of them."""
    p = G.girih_plan("7c", "f64", G.make_grid(512, 512, 512, 1), (0.4, 0.1), "mwd")
    every = G.girih_candidates(p)

    def lds(q):
        G.girih_plan_set_params(p, q)
        return G.girih_plan_info(p)[1]
    sizes = [lds(q) for q in every]
    budget = 105000   # below the double-buffered Dw = 8 stage (106080 B), above Dw = 12's single one
    G.girih_set_lds_budget(p, budget)
    kept = G.girih_candidates(p)
    assert 0 < len(kept) < len(every)
    assert all(lds(q) <= budget for q in kept)
    assert len(kept) == sum(1 for s in sizes if s <= budget)
    G.girih_set_lds_budget(p, 0)
    assert len(G.girih_candidates(p)) == len(every)
    with pytest.raises(G.GirihError) as e:
        G.girih_set_lds_budget(p, -1)
    assert e.value.code == G.E_INVALID
    G.girih_destroy(p)


def test_leapfrog_plans():
    """The second-order-in-time 25-point stencil: naive plans stream four
    domain-sized arrays (V, U read and written, C); blocked plans default to
    Dw = 16, whose B_C with N_D = 3 (the two time levels and C) is
    2*8*4*[(32 - 8) + (48 + 8)]/256 = 20 B per update in FP64."""
    g = G.make_grid(64, 48, 40, 4)
    c = (-205.0 / 24.0, 1.6, -0.2, 8.0 / 315.0, -1.0 / 560.0)
    p = G.girih_plan("25l", "f64", g, c, "naive")
    _, _, bytes_per_lup = G.girih_plan_info(p)
    assert bytes_per_lup == 32.0
    G.girih_destroy(p)
    p = G.girih_plan("25l", "f64", g, c, "mwd")
    q, _, bytes_per_lup = G.girih_plan_info(p)
    assert q["diamond_width"] == 16 and bytes_per_lup == pytest.approx(20.0)
    assert {(x["diamond_width"], x["wavefront_depth"]) for x in G.girih_candidates(p)} == {(16, 1), (8, 1)}
    G.girih_destroy(p)
    with pytest.raises(G.GirihError) as e:
        G.girih_plan("25l", "f64", g, None, "naive")          # constants are required
    assert e.value.code == G.E_INVALID


@pytest.mark.parametrize("stencil,dtype", [("7c", "f64"), ("7c", "f32"), ("25c", "f64"), ("7v", "f64"), ("7v", "f32"),
                                           ("25v", "f64"), ("25v", "f32"), ("25l", "f64"), ("25l", "f32")])
def test_plan_info_reports_the_papers_code_balance(stencil, dtype):
    """girih_plan_info gives the paper's B_C (Section "Memory traffic model")
    of the plan's diamond width, scaled to the element size, with N_D the
    field pair plus the coefficient arrays; every stencil and precision has
    a default blocked plan."""
    from oracle import models
    R = 1 if stencil.startswith("7") else 4
    nd = 2 + {"7c": 0, "7v": 7, "25c": 0, "25v": 13, "25l": 1}[stencil]
    cc = {"7c": (0.4, 0.1), "25c": (0.2, 0.05, 0.04, 0.03, 0.0133), "25l": (-8.5, 1.6, -0.2, 0.025, -0.002)}.get(stencil)
    p = G.girih_plan(stencil, dtype, G.make_grid(96, 80, 40, R), cc, "mwd")
    params, lds, bpl = G.girih_plan_info(p)
    G.girih_destroy(p)
    word = 8 if dtype == "f64" else 4
    assert bpl == pytest.approx(models.code_balance(params["diamond_width"], R, nd, word_bytes=word), rel=1e-12)


def test_wavefront_depth_plans():
    """N_F = 2 plans exist for the registered shapes: their stage holds two
    planes per row, one buffer of 51 rows x 2 x 130 FP64 values for Dw = 8
    and 128-cell rows -- the LDS that N_F = 1 spends on two stage buffers of
    one plane -- and the candidate list of a problem offers both depths."""
    g = grid(64)
    p1 = G.girih_plan("7c", "f64", g, (0.4, 0.1), "mwd", {"diamond_width": 8, "threads_x": 128})
    p2 = G.girih_plan("7c", "f64", g, (0.4, 0.1), "mwd", {"diamond_width": 8, "threads_x": 128, "wavefront_depth": 2})
    q1, lds1, _ = G.girih_plan_info(p1)
    q2, lds2, _ = G.girih_plan_info(p2)
    assert q1["wavefront_depth"] == 1 and q2["wavefront_depth"] == 2
    assert lds1 == lds2 == 51 * 2 * 130 * 8
    depths = {q["wavefront_depth"] for q in G.girih_candidates(p1)}
    assert depths == {1, 2}
    G.girih_destroy(p1)
    G.girih_destroy(p2)


def test_schedule_variant_plans():
    """Variant bit 0 (the dependency-driven schedule) and bit 1 (relaxed
    synchronisation) exist for the shapes compiled with them and are offered
    among the candidates; other shapes refuse them, and values beyond the two
    bits are invalid."""
    g = grid(64)
    for v in (1, 2, 3):
        p = G.girih_plan("7c", "f64", g, (0.4, 0.1), "mwd", {"variant": v})
        q, lds, _ = G.girih_plan_info(p)
        assert q["variant"] == v and q["diamond_width"] == 12
        # the relaxed kernels keep 32 step counters beside the stage
        assert lds == (103088 if v & 2 else 102960)
        assert {c["variant"] for c in G.girih_candidates(p)} == {0, 1, 2, 3}
        G.girih_destroy(p)
    for v in (1, 2):
        with pytest.raises(G.GirihError) as e:
            G.girih_plan("7c", "f64", g, (0.4, 0.1), "mwd", {"diamond_width": 8, "cells_per_lane": 2,
                                                             "threads_x": 64, "variant": v})
        assert e.value.code == G.E_UNSUPPORTED
    for v in (4, -1):
        with pytest.raises(G.GirihError) as e:
            G.girih_plan("7c", "f64", g, (0.4, 0.1), "mwd", {"variant": v})
        assert e.value.code == G.E_INVALID
    # FP32 7-point: the default shape (two planes per step) has both bits
    p = G.girih_plan("7c", "f32", g, (0.4, 0.1), "mwd", {"variant": 3})
    q, _, _ = G.girih_plan_info(p)
    assert q["wavefront_depth"] == 2 and q["diamond_width"] == 12
    G.girih_destroy(p)
