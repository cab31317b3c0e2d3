"""Numbers the paper prints, pinned against the benchmark's accounting (no GPU).

Sec. VI-E counts 9 FLOP per update of the 5-point star (a centre product and four fused
multiply-adds of 2 FLOP each), 10 four-byte SRAM accesses per update (arithmetic intensity about
0.23 FLOP/B), and a peak of 0.858 PFLOP/s for 700 x 700 PEs at 875 MHz, i.e. one FMA = 2 FLOP per
PE and cycle.  The benchmark's roofline uses the same convention (box49: 1 + 2 x 48 = 97 FLOP).
"""
import json
import os

import pytest

import bench

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def sec6e():
    with open(os.path.join(HERE, "golden", "sec6e_cstencil_roofline.json")) as f:
        return json.load(f)


def test_flop_per_update_matches_the_papers_count(sec6e):
    assert bench.flop_per_update(sec6e["stencil"]["taps"]) == sec6e["flop_per_update"]
    assert bench.flop_per_update(49) == 97.0 and bench.flop_per_update(9) == 17.0


def test_arithmetic_intensity_and_fma_convention(sec6e):
    ai = sec6e["flop_per_update"] / (sec6e["sram_accesses_per_update"] * sec6e["bytes_per_access"])
    assert round(ai, 2) == sec6e["arithmetic_intensity_flop_per_byte"]
    rows, cols = sec6e["pe_subarray"]
    peak = rows * cols * sec6e["clock_mhz"] * 1e6 * 2.0 / 1e15  # one FMA (2 FLOP) per PE and cycle
    assert round(peak, 3) == sec6e["peak_pflop_s"]
    # the same convention gives the MI355X vector-ALU roof the benchmark divides by
    assert bench.VALU_FP32_PEAK == pytest.approx(78.6e12, rel=1e-3)


def test_gstencil_metric():
    # Sec. VI-A: T x Nx x Ny updates in t seconds, in units of 10^9 per second
    assert bench.gstencil_s(1000, 16384, 16384, 0.41) == pytest.approx(1000 * 16384 ** 2 / 0.41 / 1e9)
    assert bench.gstencil_s(100, 512, 512, 1e-4) == pytest.approx(262.144)
