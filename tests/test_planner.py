"""Planner closed forms against the numbers the paper prints.

Sec. 7: the processor bound of Eq. (12) lies at about 1700 cores for the
2-d runs (L = 1000, D = 1, dt = 0.1, E = 0.75) and at about 320 for the 3-d
runs (L = 100, E = 0.5); slices stop working at 500 cores.  All three follow
from the pad psi = 6 sqrt(D dt) of Sec. 6.  Sec. 7.1 prints the nearest
factor pairs of 698 (2 x 349) and 1322 (2 x 661), and says such tilings
speed up roughly like a 1-d run.  Sec. 7 also reports a 1906-fold speedup
on 2700 cores, and Sec. 2.2 says the runs obey the time-step optimality
condition.  The printed values, each with its citation, are read from
golden/printed_speedup_values.json."""
import json
import math
import os

import pytest

from paper_2204_03756_amd import planner as PL

with open(os.path.join(os.path.dirname(__file__), "golden", "printed_speedup_values.json")) as f:
    G = json.load(f)
R2, R3 = G["run_parameters_2d"], G["run_parameters_3d"]
L2, L3 = R2["L"], R3["L"]
PSI = PL.pad(R2["D"], R2["dt"])


def test_pad_is_six_kernel_deviations():
    assert PSI == pytest.approx(6.0 * math.sqrt(0.1))
    with pytest.raises(ValueError):
        PL.pad(0.0, 0.1)


def test_processor_bounds_match_the_printed_values():
    b2, b3 = G["processor_bound_2d"], G["processor_bound_3d"]
    p2 = PL.max_processors(b2["efficiency"], L2, PSI, 2)
    p3 = PL.max_processors(b3["efficiency"], L3, PSI, 3)
    # "about" 1700 and 320: within 6 %; slices stop at 500 (L / psi = 527)
    assert abs(p2 - b2["about"]) / b2["about"] < 0.06
    assert abs(p3 - b3["about"]) / b3["about"] < 0.06
    assert abs(PL.slices_limit(L2, PSI) - G["slices_limit"]["cores"]) / G["slices_limit"]["cores"] < 0.06
    # the bound is where the predicted efficiency, Eq. (11), meets the threshold
    assert PL.efficiency(p2, 1000.0, PSI, 2) == pytest.approx(0.75, rel=1e-12)
    assert PL.efficiency(p3, 100.0, PSI, 3) == pytest.approx(0.5, rel=1e-12)
    # perfect squares/cubes below the bound: the 2-d runs' 40^2 = 1600 is
    # inside it and their 45^2 = 2025 is past it
    assert PL.largest_perfect_power(p2, 2) == 40 ** 2
    assert PL.largest_perfect_power(p3, 3) == 6 ** 3
    assert PL.efficiency(1600, 1000.0, PSI, 2) >= 0.75 > PL.efficiency(2025, 1000.0, PSI, 2)
    with pytest.raises(ValueError):
        PL.max_processors(1.0, 1000.0, PSI, 2)


def test_predicted_speedup_meets_the_observed_maximum():
    # Sec. 7: the 2-d runs (L = 1000) reached a 1906-fold speedup on 2700
    # cores; Eq. (10) with the same pad predicts it within 2 %, below linear
    o = G["observed_max_speedup_2d"]
    s = PL.speedup(o["cores"], L2, PSI, 2)
    assert abs(s - o["speedup"]) / o["speedup"] < 0.02
    assert s < o["cores"]
    # pads sqrt(2) narrower or twice as wide (the other readings of the
    # kernel width) miss it by far more
    for other in (PSI / math.sqrt(2.0), 2.0 * PSI):
        assert abs(PL.speedup(o["cores"], L2, other, 2) - o["speedup"]) / o["speedup"] > 0.05


def test_speedup_limits():
    # no pad: linear speedup
    assert PL.speedup(64, 1000.0, 0.0, 3) == pytest.approx(64.0)
    # one processor still counts its pad, Eq. (8) at P = 1
    assert PL.speedup(1, 1000.0, PSI, 2) == pytest.approx((1000.0 / (1000.0 + 2 * PSI)) ** 2)
    # efficiency falls with P, and the speedup tends to (L / 2 psi)^d
    es = [PL.efficiency(p, 1000.0, PSI, 2) for p in (4, 16, 64, 256, 1024)]
    assert all(a > b for a, b in zip(es, es[1:]))
    assert PL.speedup(1e12, 1000.0, PSI, 2) == pytest.approx((1000.0 / (2 * PSI)) ** 2, rel=1e-3)
    # the multi-GPU halo of 2 psi: the bound shrinks by 2^d
    assert PL.max_processors(0.75, 1000.0, 2 * PSI, 2) == pytest.approx(
        PL.max_processors(0.75, 1000.0, PSI, 2) / 4)


def test_checkerboard_factors_of_the_printed_core_counts():
    for p, f1, f2 in G["nearly_prime_factor_pairs"]["pairs"]:
        assert PL.checkerboard_factors(p, L2, L2) == (f1, f2)
    assert PL.checkerboard_factors(400, 1000.0, 1000.0) == (20, 20)
    assert PL.checkerboard_factors(1600, 1000.0, 1000.0) == (40, 40)
    assert PL.checkerboard_factors(25, 1000.0, 1000.0) == (5, 5)
    # prime counts fall back to slices (Sec. 4.2)
    assert PL.checkerboard_factors(997, 1000.0, 1000.0) == (997, 1)
    # aspect ratio: a 4:1 domain on 16 cores takes 8 x 2, the long side along x
    assert PL.checkerboard_factors(16, 4000.0, 1000.0) == (8, 2)
    assert PL.checkerboard_factors(16, 1000.0, 4000.0) == (2, 8)
    # brute force over small p: the chosen pair minimises |f2/f1 - A|
    for p in range(1, 200):
        for a in (1.0, 1.5, 3.0):
            nx, ny = PL.checkerboard_factors(p, a * 100.0, 100.0)
            assert nx * ny == p and nx >= ny
            err = abs(nx / ny - a)
            assert all(abs(max(g, p // g) / min(g, p // g) - a) >= err - 1e-12
                       for g in range(1, p + 1) if p % g == 0)


def test_tiling_speedup_reduces_to_the_closed_forms():
    box = (1000.0, 1000.0)
    for k in (1, 5, 20, 40):
        assert PL.tiling_speedup((k, k), box, PSI) == pytest.approx(PL.speedup(k * k, 1000.0, PSI, 2))
    assert PL.tiling_speedup((6, 6, 6), (100.0,) * 3, PSI) == pytest.approx(PL.speedup(216, 100.0, PSI, 3))
    # slices: the 1-d curve times the pad factor of the uncut side
    for p in (10, 100, 500):
        assert PL.tiling_speedup((p, 1), box, PSI) == pytest.approx(
            PL.speedup(p, 1000.0, PSI, 1) / (1.0 + 2 * PSI / 1000.0))
    # Sec. 7.1: nearly prime core counts fall below square tilings with fewer
    # cores, and their speedup is much closer to the 1-d curve than to the 2-d one
    bads = [p for p, _, _ in G["nearly_prime_factor_pairs"]["pairs"]]
    for bad, good in zip(bads, G["nearly_prime_factor_pairs"]["square_counts"]):
        sb = PL.tiling_speedup(PL.checkerboard_factors(bad, *box), box, PSI)
        sg = PL.tiling_speedup(PL.checkerboard_factors(good, *box), box, PSI)
        assert sb < sg
        d1 = abs(sb - PL.speedup(bad, 1000.0, PSI, 1))
        d2 = abs(sb - PL.speedup(bad, 1000.0, PSI, 2))
        assert d1 < 0.5 * d2


def test_time_step_optimality():
    # 2-d runs: N = 1e7 in L = 1000, spacing 0.316, D = 1: bound 0.05 beta <= dt = 0.1
    assert PL.dt_min(L2, R2["N"], 2, R2["D"]) == pytest.approx(0.05)
    assert PL.dt_min(L2, R2["N"], 2, R2["D"]) <= R2["dt"]
    # 3-d runs: N = 5e6 in L = 100, spacing 0.585: bound 0.171 beta, so dt = 0.1
    # meets the condition for beta <= 0.58 (the default beta = 1/2) and not at beta = 1
    s3 = 100.0 / 5e6 ** (1.0 / 3.0)
    assert PL.dt_min(100.0, 5_000_000, 3, 1.0) == pytest.approx(s3 * s3 / 2.0)
    assert PL.dt_min(100.0, 5_000_000, 3, 1.0, beta=0.5) <= 0.1 < PL.dt_min(100.0, 5_000_000, 3, 1.0)
    assert PL.dt_min(1000.0, 10_000_000, 2, 1.0, beta=0.5) <= 0.1
    with pytest.raises(ValueError):
        PL.dt_min(1.0, 0, 2, 1.0)
