"""The cost model on the host: the traffic-model features against the
paper's formulas as the oracle writes them (oracle/models.py), the variant
bits, and how proposals spread over workgroup shapes."""
import math

import numpy as np
import pytest

from oracle import models
from paper_1510_04995_amd import costmodel as C


def params(dw, tile_x, variant=0, nf=1, tx=128, vx=1):
    return {"diamond_width": dw, "wavefront_depth": nf, "tile_x": tile_x, "tile_y": dw, "tile_z": 512,
            "threads_x": tx, "threads_y": dw // 2, "variant": variant, "cells_per_lane": vx}


@pytest.mark.parametrize("stencil,dtype,dw,tile_x", [("7c", "f64", 12, 103), ("7v", "f32", 8, 86),
                                                     ("25c", "f64", 16, 40), ("25v", "f32", 16, 39)])
def test_traffic_features_follow_the_papers_model(stencil, dtype, dw, tile_x):
    R = C.RADIUS[stencil]
    f = C.features(stencil, dtype, 512, 512, 512, 64, params(dw, tile_x), 100000)
    assert len(f) == C.N_FEATURES == 22
    nd = 2 + C.STENCIL_NCOEF[stencil]
    word = 8 if dtype == "f64" else 4
    assert 2 ** f[18] == pytest.approx(models.code_balance(dw, R, nd, word_bytes=word), rel=1e-12)
    L = dw // R
    assert 2 ** f[19] == pytest.approx((tile_x + 2 * R * (L - 1)) / tile_x, rel=1e-12)


def test_launch_round_features():
    """7c FP64 on 512^3, Dw = 12 (44 diamonds in the larger row offset):
    x tile 103 gives 5 chunks, 220 workgroups, one round of the 256 CUs at
    one workgroup per CU (102960 B of LDS), filled 220/256; x tile 86 gives
    6 chunks, 264 workgroups, two rounds; a 50 KB workgroup (three per CU)
    takes 768 slots."""
    f = C.features("7c", "f64", 512, 512, 512, 64, params(12, 103), 102960)
    assert (2 ** f[20], f[21]) == (1, pytest.approx(220 / 256))
    f = C.features("7c", "f64", 512, 512, 512, 64, params(12, 86), 102960)
    assert (2 ** f[20], f[21]) == (2, pytest.approx(264 / 512))
    f = C.features("7c", "f64", 512, 512, 512, 64, params(12, 86), 50000)
    assert (2 ** f[20], f[21]) == (1, pytest.approx(264 / 768))


def test_variant_bits():
    for v, bits in ((0, (0, 0)), (1, (1, 0)), (2, (0, 1)), (3, (1, 1))):
        f = C.features("7c", "f64", 64, 64, 64, 16, params(12, 40, variant=v), 100000)
        assert (f[16], f[17]) == bits


def test_the_seven_point_default_plan_features():
    """7c FP64, Dw = 12, x tile 103 on 512^3, T = 64: B_C = 16 (22 + 26) / 144
    = 5.33 B per update, halo factor (103 + 22) / 103."""
    f = C.features("7c", "f64", 512, 512, 512, 64, params(12, 103), 102960)
    assert 2 ** f[18] == pytest.approx(16 * 48 / 144)
    assert 2 ** f[19] == pytest.approx(125 / 103)
    assert f[2] == f[3] == f[4] == 9.0 and f[15] == 6.0 and f[6] == 12.0
    assert math.isclose(f[14], 102960 / 65536)


def test_proposals_go_round_robin_over_the_shapes():
    """propose() groups candidates by workgroup shape, ranks the shapes by
    their best prediction and takes the picks round robin over them: with a
    stand-in predictor, k = 5 on a problem with more than five shapes gives
    the best-predicted tile of the five leading shapes; on the 25-point
    problem (three shapes) the best of each, then the second of the first
    two."""
    import paper_1510_04995_amd as P
    shape = lambda q: (q["diamond_width"], q["threads_x"], q["cells_per_lane"])
    m = C.CostModel.__new__(C.CostModel)      # no device: predict() replaced below

    def predict(X):
        X = np.asarray(X)
        # shapes by diamond width, wider first, then waves and cells; larger x tiles first
        return np.array([1000.0 * x[6] + 10.0 * x[11] + x[13] + 2 ** x[8] / 1000.0 for x in X])
    m.predict = predict
    sw = P.Sweep("7c", "f64", 512, 512, 512, [0.4, 0.1], "mwd")
    picks = m.propose(sw, 64, 5)
    table = C.candidate_table(sw, 64)
    assert len({shape(p) for p, _ in table}) > 5
    assert len(picks) == 5 and len({shape(q) for q in picks}) == 5
    assert [q["diamond_width"] for q in picks] == sorted((q["diamond_width"] for q in picks), reverse=True)
    for q in picks:
        assert q["tile_x"] == max(p["tile_x"] for p, _ in table if shape(p) == shape(q))
    sw.close()
    sw = P.Sweep("25c", "f64", 512, 512, 512, [0.2, 0.05, 0.04, 0.03, 0.0133], "mwd")
    table = C.candidate_table(sw, 32)
    n_shapes = len({shape(p) for p, _ in table})
    picks = m.propose(sw, 32, 5)
    shapes = [shape(q) for q in picks]
    assert n_shapes == 3 and len(picks) == 5
    assert len(set(shapes[:3])) == 3 and shapes[3] == shapes[0] and shapes[4] == shapes[1]
    sw.close()
