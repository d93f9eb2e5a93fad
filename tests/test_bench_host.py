"""Host logic of bench.py (no GPU): the algorithmic work per launch that the
roofline is priced on, the choice of bound, and the single-GPU guard."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_transfer_bytes_per_particle():
    # 2-d FP32W, one species: x 8, s 4, m 8, mask 8 in; m 8 out; jumps 8 in,
    # walked x 8, cell 4, slot 4 out = 60 B; 2.2e6 cells (rows not trimmed)
    n = 4_000_000
    assert bench.algorithmic_bytes("transfer", n, 2, 1, 4, 8, 2_220_000) == 60.0 * n
    # 3-d with trimmed rows (about 7 particles per cell): three planes of
    # masks and of recorded windows
    n3 = 2_000_000
    b3 = bench.algorithmic_bytes("transfer", n3, 3, 1, 4, 8, 287_000)
    assert b3 == (12 + 4 + 8 + 24 + 24 + 8 + 12 + 12 + 4 + 4) * n3
    # short rows (about 1.4 particles per cell): no windows
    assert bench.algorithmic_bytes("rowsum", 100, 3, 3, 4, 8, 70) == (12 + 4 + 24) * 100
    assert bench.algorithmic_bytes("scan_down", 10, 2, 1, 4, 8, 1000) == 16.0 * 1000


def test_slots_per_pair():
    # FP32W 2-d: row sum 2d + 7 per pair; transfer 2d + 13 + 3 per pair plus
    # the walk, 10 per dimension and particle
    assert bench.algorithmic_slots("rowsum", 10, 100, 2, 1, "fp32w") == 100 * 11
    assert bench.algorithmic_slots("transfer", 10, 100, 2, 1, "fp32w") == 100 * 20 + 10 * 20
    assert bench.algorithmic_slots("transfer", 10, 100, 3, 3, "fp64") == 100 * (9 + 38 + 6) + 10 * 30
    assert bench.algorithmic_slots("place", 10, 100, 2, 1, "fp32w") == 0.0


def _res(kernel_ms, pairs, ncells):
    return {"phases": {k: (ms, 1) for k, ms in kernel_ms.items()}, "pairs_per_step": pairs,
            "n_cells": ncells}


def test_roofline_takes_the_longer_ideal_time():
    n = 4_000_000
    # transfer dominant at 0.09 ms: 240 MB -> 2.67 TB/s; slots 22.6e6 x 20 + 4e6 x 20
    r = bench.roofline(_res({"transfer": 0.09, "rowsum": 0.08}, 22_600_000, 2_220_000), 2, 1, 4, 8, n)
    assert r["kernel"] == "transfer"
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(240e6 / 0.09e-3 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, rel=1e-3)
    assert r["ops_per_launch"] == 22_600_000 * 20 + n * 20
    assert r["hbm_frac"] > r["alu_frac"]
    # many pairs per particle: the VALU ideal time is the longer one
    r3 = bench.roofline(_res({"rowsum": 0.3}, 57_200_000 * 4, 287_000), 3, 1, 4, 8, 2_000_000)
    assert r3["bound"] == "alu" and r3["unit"] == "Gop/s"
    assert r3["frac"] == r3["alu_frac"] > r3["hbm_frac"]


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
