"""The cost model's candidate features on the host: the traffic-model
features against the paper's formulas as the oracle writes them
(oracle/models.py), and the variant bits."""
import math

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
    assert len(f) == C.N_FEATURES == 20
    nd = 2 + C.STENCIL_NCOEF[stencil]
    word = 8 if dtype == "f64" else 4
    assert 2 ** f[18] == pytest.approx(models.code_balance(dw, R, nd, word_bytes=word), rel=1e-12)
    L = dw // R
    assert 2 ** f[19] == pytest.approx((tile_x + 2 * R * (L - 1)) / tile_x, rel=1e-12)


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
