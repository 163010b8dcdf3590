"""Pins of the paper's analytic models (plain oracle versions) — no GPU."""
import pytest

from oracle import models
from tests.test_oracle_pins import read_golden


def test_cache_block_worked_example():
    g = read_golden("paper_models.txt")
    assert models.cache_block_bytes(8, 1, 1, 2) == g["cs_Dw8_NF1_R1_ND2"]
    # Ww = Dw + N_F - 2 enters as 2*(Dw + Ww): recover it from the example
    assert (g["cs_Dw8_NF1_R1_ND2"] - 2 * 8 * 8 / 2) / 2 - 8 == g["ww_Dw8_NF1_R1"]


def test_cache_block_values_by_hand():
    """C_S / N_xb of both equations of Section "Cache block size model",
    evaluated by hand at N_F = 1 (golden file): R = 1 for the 7-point stencils
    (N_D = 2 and 9) and R > 1 for the 25-point ones (N_D = 2 and 15)."""
    g = read_golden("paper_models.txt")
    assert models.cache_block_bytes(16, 1, 1, 2) == g["cs_Dw16_R1_ND2"]
    assert models.cache_block_bytes(32, 1, 1, 2) == g["cs_Dw32_R1_ND2"]
    assert models.cache_block_bytes(8, 1, 1, 9) == g["cs_Dw8_R1_ND9"]
    assert models.cache_block_bytes(16, 1, 1, 9) == g["cs_Dw16_R1_ND9"]
    assert models.cache_block_bytes(16, 1, 4, 2) == g["cs_Dw16_R4_ND2"]
    assert models.cache_block_bytes(32, 1, 4, 2) == g["cs_Dw32_R4_ND2"]
    assert models.cache_block_bytes(64, 1, 4, 2) == g["cs_Dw64_R4_ND2"]
    assert models.cache_block_bytes(16, 1, 4, 15) == g["cs_Dw16_R4_ND15"]
    assert models.cache_block_bytes(32, 1, 4, 15) == g["cs_Dw32_R4_ND15"]


def test_cache_block_wavefront_depth_term():
    """N_F enters the R = 1 block as N_D*Dw*(N_F-1) + 2*(N_F-1) and the R > 1
    block as N_D*Dw*(N_F-1) + 2R*(N_F-1): one more z plane of every stream
    (hand-evaluated differences, golden file)."""
    g = read_golden("paper_models.txt")
    assert models.cache_block_bytes(8, 3, 1, 2) - models.cache_block_bytes(8, 1, 1, 2) == g["cs_Dw8_R1_ND2_NF3_minus_NF1"]
    assert models.cache_block_bytes(16, 2, 4, 2) - models.cache_block_bytes(16, 1, 4, 2) == g["cs_Dw16_R4_ND2_NF2_minus_NF1"]


def test_code_balance_values():
    # Eq. for R = 1: 16*[(2Dw-2) + (N_D*Dw+2)]/Dw^2
    assert models.code_balance(16, 1, 2) == pytest.approx(16 * (30 + 34) / 256)
    assert models.code_balance(16, 1, 2) == pytest.approx(4.0)
    assert models.code_balance(8, 1, 2) == pytest.approx(8.0)
    # Eq. for R > 1: 16R*[(2Dw-2R) + (N_D*Dw+2R)]/Dw^2 ; 25c Jacobi, Dw=32 -> 8
    assert models.code_balance(32, 4, 2) == pytest.approx(8.0)
    # it tends to the streaming (N_D+2)*16*R/Dw for large Dw
    assert models.code_balance(4096, 1, 9) == pytest.approx(16 * 11 / 4096, rel=1e-3)


def test_spatial_blocking_and_flops_printed_in_paper():
    g = read_golden("paper_models.txt")
    assert models.spatial_blocking_balance("7c") == g["sb_7c"]
    assert models.spatial_blocking_balance("7c", nontemporal=True) == g["sb_7c_nt"]
    assert models.spatial_blocking_balance("7v") == g["sb_7v"]
    assert models.spatial_blocking_balance("25c-leapfrog") == g["sb_25c_leapfrog"]
    assert models.spatial_blocking_balance("25v") == g["sb_25v"]
    assert models.flops_per_lup("7c", as_written=False) == g["flops_7c"]
    assert models.flops_per_lup("7v", as_written=False) == g["flops_7v"]
    assert models.flops_per_lup("25c-leapfrog", as_written=False) == g["flops_25c_leapfrog"]
    assert models.flops_per_lup("25v", as_written=False) == g["flops_25v"]


def test_flops_as_written_count_listing_operations():
    # 7c: 4 multiplies + 3 pair sums + 3 accumulations = 10
    # 25c (Jacobi bracket): 5 multiplies + 4*5 neighbour sums + 4 accumulations = 29
    # 7v: 7 multiplies + 6 accumulations = 13 ; 25v: 13 + 12 pair sums + 12 = 37
    assert [models.flops_per_lup(s) for s in ("7c", "7v", "25c", "25v")] == [10, 13, 29, 37]


def test_diamond_volume():
    assert models.diamond_volume_per_plane(16, 1) == 128
    assert models.diamond_volume_per_plane(32, 4) == 128
