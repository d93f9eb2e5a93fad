"""Host logic of bench.py (no GPU): the algorithmic work per launch that the
roofline is priced on, the choice of bound, and the single-GPU guard."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_step_bytes_follow_the_method():
    """B = 5 d p + 4 S q + 2 s + 8 per particle-step: 172 B for the 3-d
    three-species FP32W workload, 240 B in FP64, 88 B for 2-d FP32W."""
    assert bench.step_bytes(3, 3, 4, 8) == 172.0
    assert bench.step_bytes(3, 3, 8, 8) == 240.0
    assert bench.step_bytes(2, 1, 4, 8) == 88.0


def test_static_step_is_the_transfer_alone():
    # particles that never move keep order and row sums: x read, s read,
    # masses read and written -- 2-d FP64 one species: 16 + 8 + 16 = 40 B
    assert bench.step_bytes(2, 1, 8, 8, moving=False) == 40.0
    assert bench.algorithmic_bytes("transfer", 100, 2, 1, 8, 8, 50, moving=False) == 40.0 * 100
    assert bench.algorithmic_slots("transfer", 10, 100, 2, 1, "fp32w", moving=False) == 100 * 20
    o = bench.overhead_bytes("transfer", 100, 2, 1, 8, 8, 50, moving=False)
    assert "stored_jumps" not in o and "cell_and_slot" not in o
    r = bench.roofline(_res({"transfer": 0.01}, 150_000, 2_500, 0.02), 2, 1, 8, 8, 10_000, "fp64",
                       moving=False)
    assert r["step_bytes"] == 40.0 * 10_000 and r["bytes_per_launch"] == 40.0 * 10_000


def test_kernel_shares_add_up_to_the_step():
    # the three passes' shares of the method's bytes are the whole step
    for dim, ns, tsz, msz in ((2, 1, 4, 8), (3, 3, 4, 8), (3, 3, 8, 8), (3, 1, 4, 4)):
        tot = sum(bench.algorithmic_bytes(k, 1000, dim, ns, tsz, msz, 500)
                  for k in ("place", "rowsum", "transfer"))
        assert tot == 1000 * bench.step_bytes(dim, ns, tsz, msz)
    # the transfer of the 3-d three-species FP32W workload: x 12 in, walked x
    # 12 out, s 4 in, masses 24 in and 24 out
    assert bench.algorithmic_bytes("transfer", 100, 3, 3, 4, 8, 70) == 76.0 * 100
    assert bench.algorithmic_bytes("scatter", 100, 3, 3, 4, 8, 70) == 0.0
    # implementation structures are overhead, listed apart: 3 planes of
    # neighbour bits, stored jumps, cell and slot; windows only where rows
    # are trimmed (about 7 particles per cell, not 1.4)
    o = bench.overhead_bytes("transfer", 100, 3, 3, 4, 8, 70)
    assert o == {"neighbour_bits": 2400.0, "stored_jumps": 1200.0, "cell_and_slot": 800.0}
    o7 = bench.overhead_bytes("rowsum", 700, 3, 1, 4, 8, 100)
    assert o7 == {"neighbour_bits": 700 * 24.0, "row_windows": 700 * 24.0}


def test_slots_per_pair():
    # FP32W 2-d: row sum 2d + 7 per pair; transfer 2d + 13 + 3 per pair plus
    # the walk, 10 per dimension and particle
    assert bench.algorithmic_slots("rowsum", 10, 100, 2, 1, "fp32w") == 100 * 11
    assert bench.algorithmic_slots("transfer", 10, 100, 2, 1, "fp32w") == 100 * 20 + 10 * 20
    assert bench.algorithmic_slots("transfer", 10, 100, 3, 3, "fp64") == 100 * (9 + 38 + 6) + 10 * 30
    assert bench.algorithmic_slots("place", 10, 100, 2, 1, "fp32w") == 0.0


def _res(kernel_ms, pairs, ncells, ms_per_step=1.0):
    return {"phases": {k: (ms, 1) for k, ms in kernel_ms.items()}, "pairs_per_step": pairs,
            "n_cells": ncells, "ms_per_step": ms_per_step}


def test_roofline_takes_the_longer_ideal_time():
    n = 4_000_000
    # 2-d FP32W transfer dominant at 0.09 ms: its share 2*8 + 4 + 16 = 36 B
    # per particle -> 144 MB; slots 22.6e6 x 20 + 4e6 x 20
    r = bench.roofline(_res({"transfer": 0.09, "rowsum": 0.08}, 22_600_000, 2_220_000, 0.27), 2, 1, 4, 8, n)
    assert r["kernel"] == "transfer"
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["bytes_per_launch"] == 36.0 * n
    assert r["achieved"] == pytest.approx(36.0 * n / 0.09e-3 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, rel=1e-3)
    assert r["ops_per_launch"] == 22_600_000 * 20 + n * 20
    assert r["hbm_frac"] > r["alu_frac"]
    # the whole step: 88 B per particle over 0.27 ms
    assert r["step_bytes"] == 88.0 * n
    assert r["step_frac"] == pytest.approx(88.0 * n / 0.27e-3 / 8e12, rel=1e-3)
    # many pairs per particle: the VALU ideal time is the longer one
    r3 = bench.roofline(_res({"rowsum": 0.3}, 57_200_000 * 4, 287_000), 3, 1, 4, 8, 2_000_000)
    assert r3["bound"] == "alu" and r3["unit"] == "Gop/s"
    assert r3["frac"] == r3["alu_frac"] > r3["hbm_frac"]


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_valu_issue_from_the_committed_counters():
    # the dominant kernels' VALU instructions per launch come from the
    # committed PMC summary, and only while the sources are the profiled ones
    import json
    rec = json.load(open(os.path.join(ROOT, "profiles", "valu_react3d_fp32w.json")))
    k = rec["kernels"]["rowsum"]
    v = bench.valu_issue_from_profile("rowsum", "react3d", "fp32w", k["avg_ns"] * 1e-9)
    if rec["source_sha256"] == bench.source_sha256():
        assert v == pytest.approx(k["valu_insts_per_launch"] * 4 / (1024 * 2.4e9 * k["avg_ns"] * 1e-9), rel=1e-3)
        assert 0.3 < v < 1.2
    else:
        assert v is None
    assert bench.valu_issue_from_profile("rowsum", "no_such_workload", "fp32w", 1e-3) is None
