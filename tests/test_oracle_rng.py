"""Pins of the oracle's random-walk generator (CPU only).

* Philox4x32-10 words against rocRAND's own engine run on the host (a library
  routine, not a retyping of the round function).
* The series log / sin / cos against libm within a few ulp.
* Box-Muller normals: exact special cases, moments and a KS test.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_words(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc (rocRAND headers) not available")
    exe = str(tmp_path_factory.mktemp("rr") / "rr_philox")
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950",
                    os.path.join(HERE, "helpers", "rocrand_philox_words.cpp"), "-o", exe],
                   check=True, capture_output=True)

    def run(rows):
        text = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True)
        return np.array([[int(t) for t in line.split()] for line in out.stdout.strip().splitlines()],
                        dtype=np.uint64)
    return run


def test_philox_matches_rocrand(oracle, rocrand_words):
    rng = np.random.default_rng(7)
    rows = rng.integers(0, 2**32, size=(300, 6), dtype=np.uint64)
    rows[0] = 0
    rows[1] = 2**32 - 1
    # the counters the random walk actually uses: (pid, call, step lo, step hi)
    rows[2] = [12345, 1, 99, 0, 0x54505402, 0x4D]
    ref = rocrand_words(rows)
    mine = np.array([oracle.philox4x32_10(r[:4], r[4:]) for r in rows], dtype=np.uint64)
    assert np.array_equal(mine, ref)


def test_uniform52_range_and_ends(oracle):
    assert oracle.uniform52(0, 0) == 2.0 ** -53
    assert oracle.uniform52(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    # 52 bits: the low 12 bits of the low word are dropped
    assert oracle.uniform52(0xFFF, 0) == 2.0 ** -53
    assert oracle.uniform52(0x1000, 0) == 3.0 * 2.0 ** -53
    assert oracle.uniform52(0, 1) == (2.0 * 2**20 + 1) * 2.0 ** -53


def _ulp(v):
    return math.ulp(abs(v)) if v != 0 else math.ulp(0.0)


def test_log_against_libm(oracle):
    rng = np.random.default_rng(11)
    us = np.concatenate([rng.random(20000), 10.0 ** rng.uniform(-16, 0, 5000),
                         1.0 - 10.0 ** rng.uniform(-16, -1, 2000)])
    us = us[(us > 0) & (us < 1)]
    worst = max(abs(oracle.log(float(u)) - math.log(u)) / _ulp(math.log(u)) for u in us)
    assert worst <= 2.0
    assert oracle.log(0.5) == -math.log(2.0)
    assert abs(oracle.log(2.0 ** -53) - math.log(2.0 ** -53)) <= _ulp(math.log(2.0 ** -53))


def test_sincos_against_libm(oracle):
    rng = np.random.default_rng(12)
    for u in np.concatenate([rng.random(20000), [1e-15, 0.125, 0.375, 0.5 - 1e-16, 0.999999]]):
        s, c = oracle.sincos_2pi(float(u))
        # libm's own argument 2*pi*u is rounded: |error| <= 2*pi*2^-53 ~ 7e-16
        assert abs(s - math.sin(2 * math.pi * u)) <= 1.2e-15
        assert abs(c - math.cos(2 * math.pi * u)) <= 1.2e-15
    # exact quadrant points
    assert oracle.sincos_2pi(0.25) == (1.0, -0.0)
    assert oracle.sincos_2pi(0.5) == (-0.0, -1.0)
    assert oracle.sincos_2pi(0.75) == (-1.0, 0.0)


def test_normal_pair_is_box_muller_of_philox(oracle):
    """Special case that reduces to libm: z = sqrt(-2 ln u1) (cos, sin)(2 pi u2)
    with the uniforms taken from the rocRAND-pinned Philox words."""
    for pid, call, step in [(0, 0, 0), (17, 1, 5), (2**31, 0, 2**33 + 7)]:
        seed = 0x4D54505402
        w = oracle.philox4x32_10([pid, call, step & 0xFFFFFFFF, step >> 32],
                                 [seed & 0xFFFFFFFF, seed >> 32])
        u1 = oracle.uniform52(int(w[0]), int(w[1]))
        u2 = oracle.uniform52(int(w[2]), int(w[3]))
        r = math.sqrt(-2.0 * math.log(u1))
        z = oracle.normal_pair(seed, step, pid, call)
        assert abs(z[0] - r * math.cos(2 * math.pi * u2)) <= 1e-14 * max(1.0, r)
        assert abs(z[1] - r * math.sin(2 * math.pi * u2)) <= 1e-14 * max(1.0, r)


def test_normals_moments_and_ks(oracle):
    n = 400_000
    xi = oracle.normals(20220402, 3, 3, n)
    flat = xi.ravel()
    m = flat.size
    assert abs(flat.mean()) < 5.0 / math.sqrt(m)
    assert abs(flat.var() - 1.0) < 5.0 * math.sqrt(2.0 / m)
    assert abs(stats.kurtosis(flat)) < 5.0 * math.sqrt(24.0 / m)
    for k in range(3):
        assert stats.kstest(xi[:, k], "norm").pvalue > 1e-4
    # components independent of each other and of the next step
    c = np.corrcoef(xi.T)
    assert np.all(np.abs(c - np.eye(3)) < 5.0 / math.sqrt(n))
    xi2 = oracle.normals(20220402, 4, 3, n)
    assert abs(np.corrcoef(xi[:, 0], xi2[:, 0])[0, 1]) < 5.0 / math.sqrt(n)
