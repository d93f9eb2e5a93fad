"""Benchmark: MT pair-updates/s of the MTPT step on one MI355X.

Workload: 2-d random walk + mass transfer, N = 4e6 particles uniform in
[0,2000]^2, D_RW = D_MT = 0.5, dt = 0.1, psi = 3 sqrt(4 D_MT dt), Gaussian
mass blob (sigma 50), 100 steps -- synthetic, seeded.  A "step" is one whole
MTPT step (walk, binning, row sums, transfer, totals).  The FP32-weight /
FP64-accumulation path gives ``value``; the plain FP64 path is timed beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-fp64]

Prints one JSON line.  ``roofline`` is computed for the dominant kernel from
device-side event timings of each launch and its algorithmic bytes.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz


def algorithmic_bytes(kernel: str, n: int, dim: int, ns: int, tsz: int, msz: int, ncells: int) -> float:
    """Bytes each launch must move at minimum (one read of every input it
    needs, one write of every output), per the data layout of the path."""
    pos = dim * tsz
    per = {
        "bin": pos + 4 + pos + 4 + 4,             # x, pid in; xt, cell, rank out
        "scatter": 4 + 4 + 4,                      # cell, rank in; perm out
        "cellsort": 4 + 4,                         # perm in/out (+ pid keys)
        "gather": 4 + pos + ns * msz + 4 + pos + ns * msz + 4,
        "rowsum": pos + tsz,                       # x in; s out
        "transfer": pos + tsz + ns * msz + ns * msz,  # x, s, m in; m out
    }
    if kernel in ("scan_reduce",):
        return ncells * 4.0
    if kernel in ("scan_down",):
        return ncells * 12.0
    return float(per.get(kernel, 0) * n)


def run_path(mt, W, precision: int, steps: int, warmup: int, profile_steps: int = 5):
    import torch
    w = W.rw2d(precision=precision, steps=steps)
    stream = torch.cuda.Stream()
    alloc = mt.TorchAllocator("cuda:0")
    with torch.cuda.stream(stream):
        sim = mt.Sim(w.params, w.x0, w.m0, allocator=alloc, stream=int(stream.cuda_stream))
        sim.step(warmup)
        torch.cuda.synchronize()
        st0 = sim.stats()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evs[0].record(stream)
        for k in range(steps):
            sim.step(1)
            evs[k + 1].record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st1 = sim.stats()
        per_step = sorted(evs[k].elapsed_time(evs[k + 1]) for k in range(steps))
        # per-kernel device times (separate, profiled pass)
        mt.mtpt_set_profiling(sim.h, True)
        sim.step(profile_steps)
        phases = mt.mtpt_phase_times(sim.h)
        mt.mtpt_set_profiling(sim.h, False)
        sim.close()
    pairs = st1["pairs_total"] - st0["pairs_total"]
    wall = t1 - t0
    return {
        "w": w, "pairs": int(pairs), "wall_s": wall, "value": pairs / wall,
        "ms_per_step": 1e3 * wall / steps,
        "p50_ms": per_step[len(per_step) // 2],
        "p99_ms": per_step[min(len(per_step) - 1, int(math.ceil(0.99 * len(per_step))) - 1)],
        "phases": phases, "n_cells": st1["n_cells"], "drift": st1["drift"],
        "pairs_per_step": st1["pairs_last"],
    }


def roofline(res, dim, ns, tsz, msz, n):
    phases = res["phases"]
    if not phases:
        return None
    name = max(phases, key=lambda k: phases[k][0])
    ms_total, launches = phases[name]
    avg_s = ms_total / launches / 1e3
    byt = algorithmic_bytes(name, n, dim, ns, tsz, msz, res["n_cells"])
    achieved = byt / avg_s / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "avg_launch_us": round(avg_s * 1e6, 2), "bytes_per_launch": byt,
            "phase_ms_per_step": {k: round(v[0] / v[1], 4) for k, v in phases.items()}}


def cpu_baseline(W, seconds_hint: float = 20.0):
    """The oracle on the host cores, on a bounded sample: the first steps of
    the same 4e6-particle workload (FP32 position state, as the timed path)."""
    from oracle import oracle as O
    threads = O.max_threads()
    w = W.rw2d(precision=W.FP32W_FP64ACC)
    steps = 2
    t0 = time.perf_counter()
    r = O.run(w.params, w.x0, w.m0, steps, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": float(r.pairs.sum()) / dt, "unit": "pair-updates/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"first {steps} steps of the full 4e6-particle 2-d workload, "
                      f"{int(r.pairs.sum())} pair-updates in {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the MTPT path here is single-GPU "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2204_03756_amd import mtpt, workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    mt = mtpt
    mt.load()

    r32 = run_path(mt, W, W.FP32W_FP64ACC, args.steps, args.warmup)
    w = r32["w"]
    p = w.params
    out = {
        "metric": "MT pair-updates/s on 1 GPU, FP32-comp vs FP64 path; p50/p99 sim-step latency",
        "value": r32["value"], "unit": "pair-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r32["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32-weights/f64-accum",
        "data": "synthetic (seeded uniform positions, Gaussian mass blob)",
        "config": {"workload": "rw2d: 2-d MTPT with random walk, N=4e6 in [0,2000]^2, D_RW=D_MT=0.5, "
                               "dt=0.1, psi=3*sqrt(4*D_MT*dt), 100 steps, Gaussian blob sigma 50",
                   "n": p.n, "dim": 2, "precision": "fp32w_fp64acc",
                   "pairs_per_step": r32["pairs_per_step"], "n_cells": r32["n_cells"]},
        "p50_step_ms": r32["p50_ms"], "p99_step_ms": r32["p99_ms"],
        "mass_drift": r32["drift"],
    }
    out["roofline"] = roofline(r32, 2, 1, 4, 8, p.n)
    if not args.no_fp64:
        r64 = run_path(mt, W, W.FP64, args.steps, args.warmup)
        out["fp64_path"] = {"value": r64["value"], "ms_per_step": r64["ms_per_step"],
                            "p50_step_ms": r64["p50_ms"], "p99_step_ms": r64["p99_ms"],
                            "mass_drift": r64["drift"],
                            "roofline": roofline(r64, 2, 1, 8, 8, p.n)}
        out["fp32_over_fp64"] = r32["value"] / r64["value"]
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
