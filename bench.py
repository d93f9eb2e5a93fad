"""Benchmark: MT pair-updates/s of the MTPT step on one MI355X.

Workload (the largest one that fits one GPU): 3-d random walk + mass
transfer with a bimolecular A+B->C reaction after each transfer, N = 3.2e7
particles uniform in [0,318]^3, D_RW = 0.3, D_MT = 0.7, dt = 0.05,
psi = 3 sqrt(4 D_MT dt), three species (A = 1 for x < 159, B = 1 for
x >= 159, C = 0), k = 1 -- synthetic, seeded.  A "step" is one whole MTPT
step (walk, binning, row sums, transfer, reaction, totals).  The
FP32-weight / FP64-accumulation path gives ``value``; the plain FP64 path is
timed beside it.  A short serving mix (closed loop, then Poisson arrivals)
is reported under ``serving``.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--no-cpu] [--no-fp64] [--no-serve]

Workloads: react3d (the default and the benchmark line), rw2d, rw3d, adv2d, aniso2d, plain2d (the
latency-bound 1e4-particle static workload, whose figures are the step p50/p99), serve (the
serving mix alone).

Prints one JSON line.  ``roofline`` prices the dominant kernel on its share
of the method's algorithmic bytes (device-side event timings of each
launch), and the whole step on the method's bytes per particle-step
(``step_frac``).
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
VALU_PEAK_GOPS = 256 * 64 * 2.4e9 / 1e9    # VALU lane-slots/s: 256 CUs x 64 lanes x 2.4 GHz


def step_bytes(dim: int, ns: int, tsz: int, msz: int, moving: bool = True) -> float:
    """Algorithmic HBM bytes per particle and step of the whole method, with
    the walk fused into the transfer pass: positions p = tsz bytes per
    coordinate, masses q = msz per species, row sums s = tsz, pid 4:
    B = 5 d p + 4 S q + 2 s + 8 (positions read and written by the sort, read
    by the row sums, read by the transfer and written walked; masses read and
    written by the sort and by the transfer; row sums written and read; pid
    read and written by the sort).  Particles that never move keep their
    order and their row sums, so a step of such a sim is the transfer alone:
    B = d p + s + 2 S q."""
    if not moving:
        return dim * tsz + tsz + 2.0 * ns * msz
    return 5.0 * dim * tsz + 4.0 * ns * msz + 2.0 * tsz + 8.0


def algorithmic_bytes(kernel: str, n: int, dim: int, ns: int, tsz: int, msz: int, ncells: int,
                      moving: bool = True) -> float:
    """The kernel's share of the method's bytes (step_bytes), per launch:
    place   the sort: positions, masses and pid read and written (2dp + 2Sq + 8)
    rowsum  positions read, row sums written (dp + s)
    transfer positions and row sums read, masses read and written, walked
            positions written (2dp + s + 2Sq; dp + s + 2Sq when the
            particles do not move)
    The shares add up to step_bytes; every other kernel (histogram scan,
    scatter, finalize) and every other byte (neighbour bits, recorded
    windows, stored jumps, cell ids and slots, halo re-reads) is overhead of
    this implementation (overhead_bytes)."""
    pos = dim * tsz
    share = {
        "place": 2 * pos + 2 * ns * msz + 8,
        "rowsum": pos + tsz,
        "transfer": (2 if moving else 1) * pos + tsz + 2 * ns * msz,
    }
    return float(share.get(kernel, 0) * n)


def overhead_bytes(kernel: str, n: int, dim: int, ns: int, tsz: int, msz: int, ncells: int,
                   moving: bool = True) -> dict:
    """Bytes a launch moves beyond its algorithmic share, by structure (one
    read or write each; the measured traffic adds halo re-reads and partial
    cache lines)."""
    planes = 3 if dim == 3 else 1
    masks = 8 * planes                             # neighbour bits per particle and plane
    # recorded x-windows per particle and plane, where the library trims rows
    # (rows of three cells holding 12 or more particles on average)
    wins = masks if ncells > 0 and 3.0 * n / ncells >= 12.0 else 0
    pos = dim * tsz
    per = {
        "rowsum": {"neighbour_bits": masks, "row_windows": wins},
        "transfer": ({"neighbour_bits": masks, "row_windows": wins, "stored_jumps": pos,
                      "cell_and_slot": 8} if moving else {"neighbour_bits": masks, "row_windows": wins}),
        "place": {"perm": 4, "cell_offsets": 8, "stored_jumps": pos},
        "scatter": {"cell_and_slot": 8, "perm": 4},
    }.get(kernel, {})
    out = {k: float(v * n) for k, v in per.items() if v}
    if kernel == "scan_reduce":
        out = {"cell_counts": ncells * 8.0}
    elif kernel == "scan_down":
        out = {"cell_counts_and_offsets": ncells * 16.0}
    return out


def run_path(mt, W, precision: int, steps: int, warmup: int, profile_steps: int = 5,
             workload: str = "rw2d", n=None):
    import torch
    w = W.make(workload, precision=precision, steps=steps, **({"n": n} if n else {}))
    stream = torch.cuda.Stream()
    alloc = mt.TorchAllocator("cuda:0")
    with torch.cuda.stream(stream):
        tc0 = time.perf_counter()
        sim = mt.Sim(w.params, w.x0, w.m0, allocator=alloc, stream=int(stream.cuda_stream))
        torch.cuda.synchronize()
        create_s = time.perf_counter() - tc0
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
        "pairs_per_step": st1["pairs_last"], "create_s": create_s,
    }


# Algorithmic VALU lane-slots (one slot = one lane of one VALU instruction at
# the issue rate: FP32 without packing and FP64 alike; transcendentals count
# 4), per ordered pair within psi and per particle, of the two ALU-bound
# passes:
#   rowsum   r^2 (2d), cutoff test, scale, exp (4), add            = 2d + 7
#   transfer the same K (2d + 6), W = 2K rcp(s_i + s_j) (7), and per
#            species the increment (FP32W: FP64 sub, cvt, FP64 fma = 3;
#            Kahan: 6 FP32 ops)                                     = 2d + 13 + c S
#   FP64     rowsum: canonical r^2 (3d - 1), test, exp (~25), add  = 3d + 26
#            transfer: the same K, W with an FP64 divide (~12), per
#            species sub and fma (2)                                = 3d + 38 + 2 S
#   walk     per particle in the transfer pass: jump add, reflection test
#            and cell index, 10 per dimension (the generator runs in the
#            place pass)
def algorithmic_slots(kernel: str, n: int, pairs: int, dim: int, ns: int, prec: str,
                      moving: bool = True) -> float:
    walk = 10.0 * dim if moving else 0.0
    if kernel == "rowsum":
        per = 3 * dim + 26.0 if prec == "fp64" else 2 * dim + 7.0
        return pairs * per
    if kernel == "transfer":
        if prec == "fp64":
            per = 3 * dim + 38.0 + 2.0 * ns
        else:
            per = 2 * dim + 13.0 + {"fp32w": 3.0, "kahan": 6.0}[prec] * ns
        return pairs * per + n * walk
    return 0.0


def roofline(res, dim, ns, tsz, msz, n, prec="fp32w", moving=True):
    """The dominant kernel against both rooflines (bound: the one with the
    longer ideal time), plus the whole step on the method's bytes."""
    phases = res["phases"]
    if not phases:
        return None
    name = max(phases, key=lambda k: phases[k][0])
    ms_total, launches = phases[name]
    avg_s = ms_total / launches / 1e3
    common = {"kernel": name, "avg_launch_us": round(avg_s * 1e6, 2),
              "phase_ms_per_step": {k: round(v[0] / v[1], 4) for k, v in phases.items()}}
    byt = algorithmic_bytes(name, n, dim, ns, tsz, msz, res["n_cells"], moving)
    hbm = byt / avg_s / 1e9
    out = {**common, "bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(hbm / HBM_PEAK_GBS, 4), "traffic": None, "bytes_per_launch": byt,
           "overhead_bytes_per_launch": overhead_bytes(name, n, dim, ns, tsz, msz, res["n_cells"], moving)}
    if name in ("rowsum", "transfer"):
        slots = algorithmic_slots(name, n, res["pairs_per_step"], dim, ns, prec, moving)
        alu = slots / avg_s / 1e9
        out["ops_per_launch"] = slots
        out["alu_frac"] = round(alu / VALU_PEAK_GOPS, 4)
        out["hbm_frac"] = round(hbm / HBM_PEAK_GBS, 4)
        if alu / VALU_PEAK_GOPS > hbm / HBM_PEAK_GBS:
            out.update({"bound": "alu", "achieved": round(alu, 1), "peak": VALU_PEAK_GOPS,
                        "unit": "Gop/s", "frac": round(alu / VALU_PEAK_GOPS, 4)})
    # the whole step: the method's bytes per particle-step over the step time
    sb = step_bytes(dim, ns, tsz, msz, moving) * n
    step_s = res["ms_per_step"] / 1e3
    out["step_bytes"] = sb
    out["step_bytes_per_particle"] = step_bytes(dim, ns, tsz, msz, moving)
    out["step_achieved_gbs"] = round(sb / step_s / 1e9, 1)
    out["step_frac"] = round(sb / step_s / 1e9 / HBM_PEAK_GBS, 4)
    return out


def source_sha256() -> str:
    """sha256 over the library's sources (kernels, headers, runtime), in name order."""
    import hashlib
    d = os.path.join(ROOT, "paper_2204_03756_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def traffic_from_profile(kernel: str, workload: str, precision: str):
    """HBM bytes per launch of a kernel from the committed PMC summary, or
    None when the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    sha = source_sha256()
    k = rec.get("kernels", {}).get(kernel)
    if rec.get("source_sha256") != sha or k is None:
        return None
    return k["bytes_per_launch"]


def valu_issue_from_profile(kernel: str, workload: str, precision: str, avg_s: float):
    """Measured VALU issue of a kernel: its VALU instructions per launch
    (SQ_INSTS_VALU from the committed PMC summary) x 4 cycles (a wave64
    instruction on a 16-lane SIMD) over the cycles of 1024 SIMDs at 2.4 GHz
    during the launch time measured here; None when the kernel source changed
    since the counters were taken or no summary covers the workload."""
    path = os.path.join(ROOT, "profiles", f"valu_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    k = rec.get("kernels", {}).get(kernel)
    if rec.get("source_sha256") != source_sha256() or k is None or avg_s <= 0:
        return None
    return round(k["valu_insts_per_launch"] * 4.0 / (1024 * 2.4e9 * avg_s), 4)


def profile_driver(mt, W, workload: str, precision: int, steps: int):
    """Target of the PMC runs: a calibration copy of a known size, then a few
    steps of one workload.  Prints nothing but its own markers."""
    import torch
    n = 64 * 1024 * 1024                           # 256 MiB of float32
    x = torch.ones(n, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"calibration copy: {4 * n} bytes read and written per launch", flush=True)
    w = W.make(workload, precision=precision, steps=steps)
    sim = mt.Sim(w.params, w.x0, w.m0, allocator=mt.TorchAllocator("cuda:0"))
    sim.step(steps)
    st = sim.stats()
    sim.close()
    print(f"profiled {workload} precision {precision}: {steps} steps, pairs/step {st['pairs_last']}",
          flush=True)


def cpu_baseline(W, workload: str = "react3d", steps: int = 1, n=None, target_s: float = 10.0):
    """The oracle on the host cores, on a bounded sample: the first step(s)
    of the same workload (FP32 position state, as the timed path) -- one
    step, or as many as take about target_s seconds when one step is
    quicker than half of that (at most the workload's own steps)."""
    from oracle import oracle as O
    threads = O.max_threads()
    w = W.make(workload, precision=W.FP32W_FP64ACC, **({"n": n} if n else {}))
    if w.params.n <= 100_000:
        steps = w.steps                            # a small workload runs whole
    t0 = time.perf_counter()
    r = O.run(w.params, w.x0, w.m0, steps, threads=threads)
    dt = time.perf_counter() - t0
    if dt < 0.5 * target_s and steps < w.steps:
        steps = min(w.steps, max(steps + 1, int(math.ceil(target_s / (dt / steps)))))
        t0 = time.perf_counter()
        r = O.run(w.params, w.x0, w.m0, steps, threads=threads)
        dt = time.perf_counter() - t0
    p = w.params
    parts = (["walk"] if p.d_rw > 0.0 or any(v != 0.0 for v in p.vel) else []) + \
        ["K-D tree search", "transfer"] + (["reaction"] if p.k_react > 0.0 else [])
    which = f"all {steps} steps" if steps == w.steps else f"first {steps} step(s)"
    return {"value": float(r.pairs.sum()) / dt, "unit": "pair-updates/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{which} of the {p.n:.3g}-particle {workload} workload "
                      f"({', '.join(parts)}), {int(r.pairs.sum())} pair-updates "
                      f"in {dt:.1f} s on {threads} threads"}


def serve_bench(mt, W, n_req: int, seed: int = 20220404, budget: int = 0):
    """The serving mix: closed-loop capacity first (all requests at t = 0),
    then a Poisson stream at 80 % of that capacity, both through the pool
    (budget: its HBM bytes, 0 for 90 % of the free memory)."""
    from paper_2204_03756_amd import serve
    import torch
    alloc = mt.TorchAllocator("cuda:0")
    reqs = [W.request(i, base_seed=seed) for i in range(n_req)]
    be = serve.PoolBackend(budget, 64, allocator=alloc)
    try:
        closed = serve.serve(be, reqs, None, realtime=True).summary()
    finally:
        be.close()
    torch.cuda.synchronize()
    rate = 0.8 * closed["sims_per_s"]
    reqs2 = [W.request(n_req + i, base_seed=seed) for i in range(n_req)]
    arr = W.arrivals(n_req, rate, seed=seed + 1)
    be = serve.PoolBackend(budget, 64, allocator=alloc)
    try:
        open_ = serve.serve(be, reqs2, arr, realtime=True).summary()
    finally:
        be.close()
    return closed, open_, rate


SERVE_TEXT = ("serve: Poisson stream of independent 2-d/3-d sims, N log-uniform in [1e4,1e6], density 1, "
              "D in {0.5,1,2} (D_RW = D_MT = D/2), 20-200 steps, Kahan FP32, admitted by free HBM; "
              "closed loop first, then arrivals at 0.8x its capacity")

WORKLOAD_TEXT = {
    "rw2d": "rw2d: 2-d MTPT with random walk, N=4e6 in [0,2000]^2, D_RW=D_MT=0.5, dt=0.1, "
            "psi=3*sqrt(4*D_MT*dt), 100 steps, Gaussian blob sigma 50",
    "rw3d": "rw3d: 3-d MTPT with random walk, N=2e6 in [0,126]^3, D_RW=D_MT=1, dt=0.1, "
            "psi=3*sqrt(4*D_MT*dt), 100 steps, 1000-particle central source",
    "react3d": "react3d: 3-d MTPT, N=3.2e7 in [0,318]^3, D_RW=0.3, D_MT=0.7, dt=0.05, 200 steps, "
               "A+B->C mass-based reaction after each transfer, k=1",
    "adv2d": "adv2d: rw2d with a drift velocity v=(1, 0.5) (advection-dispersion), N=4e6 in "
             "[0,2000]^2, 100 steps",
    "plain2d": "plain2d: 2-d MTPT, pure mass transfer (no random walk), N=1e4 in [0,100]^2, D_MT=1, "
               "dt=0.1, psi=3*sqrt(4*D_MT*dt), 50 steps, m=1 for x<50 else 0 (latency-bound: the "
               "step p50/p99 are its figures)",
    "aniso2d": "aniso2d: rw2d with a rotated dispersion tensor (principal values 2D and D/2, axes at "
               "30 degrees; walk and mass "
               "transfer), N=4e6 in [0,2000]^2, 100 steps",
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--workload", default="react3d",
                    choices=["react3d", "rw2d", "rw3d", "adv2d", "aniso2d", "plain2d", "serve"],
                    help="react3d (the largest single-GPU workload) is the benchmark line; the "
                         "others are reported the same way")
    ap.add_argument("--n", type=int, default=None,
                    help="particles (default: the workload's own size); the box is scaled to keep "
                         "the workload's density, e.g. --n 4170000 for one GPU's share of the 3-d "
                         "reacting workload split over eight")
    ap.add_argument("--requests", type=int, default=120, help="serving mix size (--workload serve)")
    ap.add_argument("--serve-requests", type=int, default=48, help="serving mix size on the benchmark line")
    ap.add_argument("--budget-mb", type=int, default=0,
                    help="HBM budget of the serving pool in MiB (--workload serve; 0: 90 %% of free memory)")
    ap.add_argument("--profile-driver", action="store_true",
                    help="run a calibration copy and a few steps (for rocprofv3 --pmc)")
    ap.add_argument("--precision", default="fp32w", choices=["fp64", "fp32w", "kahan"])
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

    if args.profile_driver:
        profile_driver(mt, W, args.workload, W.PRECISIONS[args.precision], args.steps)
        return

    if args.workload == "serve":
        closed, open_, rate = serve_bench(mt, W, args.requests, budget=args.budget_mb << 20)
        print(json.dumps({
            "metric": "serving mix: sims/s and p50/p99 request latency (continuous batching)",
            "value": open_["sims_per_s"], "unit": "sims/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f32-kahan", "data": "synthetic",
            "config": {"workload": SERVE_TEXT, "requests": args.requests, "poisson_rate_per_s": rate,
                       "hbm_budget_mib": args.budget_mb or None},
            "closed_loop": closed, "poisson": open_}), flush=True)
        return

    workload = args.workload
    r32 = run_path(mt, W, W.FP32W_FP64ACC, args.steps, args.warmup, workload=workload, n=args.n)
    print(f"fp32w path: {r32['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    w = r32["w"]
    p = w.params
    out = {
        "metric": "MT pair-updates/s on 1 GPU, FP32-comp vs FP64 path; p50/p99 sim-step latency",
        "value": r32["value"], "unit": "pair-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r32["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32-weights/f64-accum",
        "data": "synthetic (seeded uniform positions, workload's initial masses)",
        "config": {"workload": WORKLOAD_TEXT[workload] + (
                       f" -- scaled to N={p.n} at the same density" if args.n else ""),
                   "n": p.n, "dim": p.dim, "species": p.n_species, "precision": "fp32w_fp64acc",
                   "pairs_per_step": r32["pairs_per_step"], "n_cells": r32["n_cells"]},
        "create_s_pcie_inclusive": r32["create_s"],
        "p50_step_ms": r32["p50_ms"], "p99_step_ms": r32["p99_ms"],
        "mass_drift": r32["drift"],
    }
    ns = p.n_species
    moving = p.d_rw > 0.0 or any(v != 0.0 for v in p.vel)
    out["roofline"] = roofline(r32, p.dim, ns, 4, 8, p.n, "fp32w", moving)
    if out["roofline"] and not args.n:
        rf32 = out["roofline"]
        rf32["traffic"] = traffic_from_profile(rf32["kernel"], workload, "fp32w")
        rf32["valu_issue_frac"] = valu_issue_from_profile(rf32["kernel"], workload, "fp32w",
                                                          rf32["avg_launch_us"] * 1e-6)
    if workload == "rw3d":
        rk = run_path(mt, W, W.FP32_KAHAN, args.steps, args.warmup, workload=workload, n=args.n)
        rfk = roofline(rk, p.dim, ns, 4, 4, p.n, "kahan", moving)
        if rfk and not args.n:
            rfk["traffic"] = traffic_from_profile(rfk["kernel"], workload, "kahan")
        out["kahan_path"] = {"value": rk["value"], "ms_per_step": rk["ms_per_step"],
                             "p50_step_ms": rk["p50_ms"], "p99_step_ms": rk["p99_ms"],
                             "mass_drift": rk["drift"], "roofline": rfk}
    if not args.no_fp64:
        r64 = run_path(mt, W, W.FP64, args.steps, args.warmup, workload=workload, n=args.n)
        print(f"fp64 path: {r64['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
        rf = roofline(r64, p.dim, ns, 8, 8, p.n, "fp64", moving)
        if rf and not args.n:
            rf["traffic"] = traffic_from_profile(rf["kernel"], workload, "fp64")
        out["fp64_path"] = {"value": r64["value"], "ms_per_step": r64["ms_per_step"],
                            "p50_step_ms": r64["p50_ms"], "p99_step_ms": r64["p99_ms"],
                            "mass_drift": r64["drift"], "roofline": rf}
        out["fp32_over_fp64"] = r32["value"] / r64["value"]
    if not args.no_serve:
        closed, open_, rate = serve_bench(mt, W, args.serve_requests)
        print(f"serving: {open_['sims_per_s']:.1f} sims/s", file=sys.stderr, flush=True)
        out["serving"] = {"workload": SERVE_TEXT, "requests": args.serve_requests,
                          "closed_loop": closed, "poisson": {**open_, "rate_per_s": rate}}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(W, workload, n=args.n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
