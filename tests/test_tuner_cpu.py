"""The tuner's search and adaptive test length (paper, Section "Auto-tuning")
on fake measurement backends, through the C ABI (girih_tune_search,
girih_adaptive_time run the same code as girih_tune; no GPU needed).

The fake cost surface is convex per thread shape (the paper remarks that the
tuning space it searched is convex), so hill climbing must reach each shape's
optimum and the overall optimum with fewer measurements than the exhaustive
search."""
import itertools

import pytest

from paper_1510_04995_amd import girih as G


def candidates(nfs=(1,)):
    out = []
    for (tx, vx), dw, nf in itertools.product([(128, 1), (64, 2), (192, 1)], (4, 8, 12, 16, 20), nfs):
        for tile in (40, 56, 72, 88, 103):
            if tile > 140 - 5 * dw:
                continue
            out.append({"diamond_width": dw, "wavefront_depth": nf, "tile_x": tile, "threads_x": tx,
                        "cells_per_lane": vx, "threads_y": dw // 2})
    return out


def surface(p):
    """Convex in (diamond width, depth, x tile) per shape, optimum inside."""
    shape_best = {(128, 1): 600.0, (64, 2): 640.0, (192, 1): 580.0}[(p["threads_x"], p["cells_per_lane"])]
    dw_opt = {(128, 1): 12, (64, 2): 8, (192, 1): 16}[(p["threads_x"], p["cells_per_lane"])]
    tile_opt = 140 - 5 * p["diamond_width"] - 10
    return (shape_best - 3.0 * (p["diamond_width"] - dw_opt) ** 2 - 0.02 * (p["tile_x"] - tile_opt) ** 2
            - 25.0 * (p["wavefront_depth"] - 2) ** 2)


def test_exhaustive_measures_every_candidate_once():
    cands = candidates()
    seen = []
    bi, bg, n = G.girih_tune_search(cands, "exhaustive", lambda p: seen.append(p) or surface(p))
    assert n == len(cands) == len(seen)
    best = max(range(len(cands)), key=lambda i: surface(cands[i]))
    assert bi == best and bg == pytest.approx(surface(cands[best]))


@pytest.mark.parametrize("nfs", [(1,), (1, 2, 3)])
def test_hill_climbing_reaches_the_optimum_with_fewer_measurements(nfs):
    cands = candidates(nfs)
    seen = []
    bi, bg, n = G.girih_tune_search(cands, "hillclimb", lambda p: seen.append(tuple(sorted(p.items()))) or surface(p))
    best = max(range(len(cands)), key=lambda i: surface(cands[i]))
    assert bi == best
    assert n == len(seen) == len(set(seen)) < len(cands)
    # every shape was searched: its own optimum was measured
    for shape in {(c["threads_x"], c["cells_per_lane"]) for c in cands}:
        group = [c for c in cands if (c["threads_x"], c["cells_per_lane"]) == shape]
        top = max(group, key=surface)
        assert tuple(sorted({**top, "variant": 0, "tile_y": 0, "tile_z": 0}.items())) in seen


def test_hill_climbing_stops_at_a_local_optimum():
    # a surface with two bumps along the diamond width: the climb from the
    # median width stays on its own bump
    cands = [c for c in candidates() if c["threads_x"] == 128]
    def bumpy(p):
        return {4: 300, 8: 280, 12: 290, 16: 285, 20: 500}[p["diamond_width"]] + 0.01 * p["tile_x"]
    bi, bg, n = G.girih_tune_search(cands, "hillclimb", bumpy)
    assert cands[bi]["diamond_width"] == 12 and n < len(cands)
    ex_i, ex_g, ex_n = G.girih_tune_search(cands, "exhaustive", bumpy)
    assert cands[ex_i]["diamond_width"] == 20 and ex_n == len(cands) and ex_g >= bg


def test_failed_candidates_are_skipped():
    cands = candidates()[:6]
    bi, bg, n = G.girih_tune_search(cands, "model", lambda p: 0.0 if p["diamond_width"] == 4 else p["tile_x"])
    assert n == 6 and cands[bi]["diamond_width"] != 4
    bi, bg, n = G.girih_tune_search(cands, "model", lambda p: -1.0)
    assert bi == -1 and n == 6


def test_adaptive_length_doubles_until_long_enough_and_stable():
    calls = []
    pers = iter([0.008, 0.006, 0.005, 0.0045, 0.004, 0.004, 0.004])
    def timer(reps):
        calls.append(reps)
        return reps * next(pers)
    per, reps, tries = G.girih_adaptive_time(timer, tol=0.03, min_seconds=0.05)
    # the run count doubles while a measurement lasts under 50 ms (1, 2, 4, 8
    # runs), then stays (16 runs = 64 ms); two consecutive per-run times
    # within 3 % end it
    assert calls == [1, 2, 4, 8, 16, 16]
    assert per == pytest.approx(0.004) and reps == 16 and tries == 6


def test_adaptive_length_keeps_length_once_long_enough():
    calls = []
    seq = iter([0.1, 0.2, 0.13, 0.1, 0.1])
    def timer(reps):
        calls.append(reps)
        return reps * next(seq)
    per, reps, tries = G.girih_adaptive_time(timer, tol=0.03, min_seconds=0.05)
    assert calls == [1, 1, 1, 1, 1] and per == pytest.approx(0.1) and tries == 5


def test_adaptive_length_gives_up_after_max_tries():
    calls = []
    def timer(reps):
        calls.append(reps)
        return reps * (0.1 if len(calls) % 2 else 0.12)   # never within 3 %
    per, reps, tries = G.girih_adaptive_time(timer, tol=0.03, min_seconds=0.05, max_tries=7)
    assert tries == 7 and len(calls) == 7


def test_adaptive_length_reports_a_failed_run():
    with pytest.raises(G.GirihError) as e:
        G.girih_adaptive_time(lambda reps: -1.0)
    assert e.value.code == G.E_HIP
