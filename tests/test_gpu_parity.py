"""GPU parity of the HIP path against the CPU oracle, through the C-ABI.

Bars (normwise error per species, max_i |m_i - o_i| / max_i |o_i|):
  FP64 path 1e-12, FP32W_FP64ACC and FP32_KAHAN 1e-5.
Positions (the random walk) and neighbour sets are compared bit for bit; the
per-step pair counts exactly.  Sizes span many 256-particle blocks, many scan
tiles and a ragged tail.
"""
import math
import os
import sys

import numpy as np
import pytest

from paper_2204_03756_amd import workloads as W

pytestmark = pytest.mark.gpu

from gpu_helpers import (PREC_NAMES, TOL, check_parity, gpu_run, load_mt, normwise,  # noqa: E402
                         oracle_run, say)


@pytest.fixture(scope="module")
def mt():
    return load_mt()


# ----------------------------------------------------------------- parity --
@pytest.mark.parametrize("prec", [W.FP64, W.FP32W_FP64ACC, W.FP32_KAHAN])
def test_plain2d_config(mt, oracle, prec):
    """Pure mass transfer, 1e4 particles, 50 steps (the full plain 2-d workload)."""
    w = W.plain2d(precision=prec)
    check_parity(mt, oracle, w, w.steps)


@pytest.mark.parametrize("prec", [W.FP64, W.FP32W_FP64ACC, W.FP32_KAHAN])
def test_rw2d_small(mt, oracle, prec):
    w = W.rw2d(n=40_000 + 37, steps=10, precision=prec)
    check_parity(mt, oracle, w, w.steps)


@pytest.mark.parametrize("prec", [W.FP64, W.FP32W_FP64ACC, W.FP32_KAHAN])
def test_rw3d_small(mt, oracle, prec):
    w = W.rw3d(n=30_000 + 101, steps=8, precision=prec, n_src=50)
    check_parity(mt, oracle, w, w.steps)


@pytest.mark.parametrize("case,prec", [("rw2d", W.FP32W_FP64ACC), ("rw3d", W.FP64),
                                       ("react3d", W.FP32W_FP64ACC), ("plain2d", W.FP64)])
def test_throughput_tile_shape_at_small_sizes(mt, oracle, monkeypatch, case, prec):
    """The tile shapes large sims get (MTPT_MIN_TILES=1: no minimum tile
    count), on sims small enough for the oracle that would otherwise be cut
    into at least 256 tiles."""
    monkeypatch.setenv("MTPT_MIN_TILES", "1")
    w = {"rw2d": lambda: W.rw2d(n=40_000 + 37, steps=6, precision=prec),
         "rw3d": lambda: W.rw3d(n=30_000 + 101, steps=5, precision=prec, n_src=50),
         "react3d": lambda: W.react3d(n=40_000 + 3, steps=4, precision=prec),
         "plain2d": lambda: W.plain2d(n=20_000, steps=20, precision=prec)}[case]()
    say(f"  throughput tile shape {case} {PREC_NAMES[prec]} n={w.params.n}")
    m1, x1, st1, _ = check_parity(mt, oracle, w, w.steps)
    # the tile shape changes neither positions nor masses nor pair counts
    monkeypatch.setenv("MTPT_MIN_TILES", "256")
    m2, x2, st2 = gpu_run(mt, w, w.steps)
    assert np.array_equal(m1, m2) and np.array_equal(x1, x2)
    assert st1["pairs_total"] == st2["pairs_total"]


@pytest.mark.parametrize("prec", [W.FP64, W.FP32W_FP64ACC, W.FP32_KAHAN])
def test_react3d_small(mt, oracle, prec):
    w = W.react3d(n=20_000 + 3, steps=6, precision=prec)
    m, x, st, ref = check_parity(mt, oracle, w, w.steps)
    # invariants of the reaction on the GPU result: A - B unchanged per
    # particle by the reaction, totals A + C and B + C kept by the transfer
    ta = m[0].sum() + m[2].sum()
    tb = m[1].sum() + m[2].sum()
    tol = 1e-9 if prec != W.FP32_KAHAN else 1e-4
    assert abs(ta - w.m0[0].sum()) <= tol * w.m0[0].sum()
    assert abs(tb - w.m0[1].sum()) <= tol * w.m0[1].sum()
    assert m[2].sum() > 0


# ------------------------------------------------------ neighbour sets ----
@pytest.mark.parametrize("dim,prec", [(2, W.FP64), (2, W.FP32W_FP64ACC), (3, W.FP64), (3, W.FP32_KAHAN)])
def test_neighbors_bit_exact(mt, oracle, dim, prec):
    w = W.rw2d(n=20_000, steps=3, precision=prec) if dim == 2 else \
        W.rw3d(n=20_000, steps=3, precision=prec, n_src=20)
    alloc = mt.TorchAllocator("cuda:0")
    say(f"  neighbours dim={dim} prec={PREC_NAMES[prec]}")
    with mt.Sim(w.params, w.x0, w.m0, allocator=alloc) as sim:
        row0, col0 = sim.neighbors()
        sim.step(3)
        row3, col3 = sim.neighbors()
    x0 = w.x0 if prec == W.FP64 else w.x0.astype(np.float32).astype(np.float64)
    orow, ocol = oracle.neighbors(x0, w.params.psi_eff, "brute")
    assert np.array_equal(row0, orow) and np.array_equal(col0, ocol)
    ref = oracle_run(oracle, w, 3)
    orow, ocol = oracle.neighbors(ref.x, w.params.psi_eff, "kdtree")
    assert np.array_equal(row3, orow) and np.array_equal(col3, ocol)


def _hot_sets(mt, w, steps):
    """Positions and the pairs the last step's row-sum and transfer passes used."""
    alloc = mt.TorchAllocator("cuda:0")
    with mt.Sim(w.params, w.x0, w.m0, allocator=alloc) as sim:
        sim.step(steps)
        x = sim.positions()
        return x, sim.step_neighbors(0), sim.step_neighbors(1)


def _dense3d(n, density, prec):
    L = (n / density) ** (1.0 / 3.0)
    p = W.Params(dim=3, n=n, lo=[0.0, 0.0, 0.0], hi=[L, L, L], d_rw=1.0, d_mt=1.0, dt=0.1, beta=0.5,
                 psi=0.0, seed=0x4D5450540D, precision=prec)
    rng = np.random.Generator(np.random.Philox(20221203))
    x = rng.random((n, 3)) * L
    m = (x[:, 0] < L / 2).astype(np.float64)[None, :]
    return W.Workload(f"dense3d-rho{density}", p, x, m, 2, {})


def _ramp3s(prec):
    """Three species, A+B->C, particle density rising 10-fold along x (0.3 to 3
    times the mean of 1): the row-sum and transfer passes tile the grid
    differently (positions only, against positions, row sums and three
    species), so where the density crosses their LDS capacities some
    particles' row-sum tiles overflow (no recorded neighbours) while their
    transfer tiles are staged, and the reverse."""
    lx, ly, lz = 60.0, 30.0, 30.0
    n = int(lx * ly * lz * 1.65)
    p = W.Params(dim=3, n=n, lo=[0.0, 0.0, 0.0], hi=[lx, ly, lz], d_rw=0.3, d_mt=0.7, dt=0.05,
                 beta=0.5, psi=0.0, k_react=1.0, n_species=3, seed=0x4D5450541D, precision=prec)
    rng = np.random.Generator(np.random.Philox(20221205))
    # x from the density 0.3 + 2.7 u (u = x / lx) by its inverse distribution
    a, b = 0.3, 2.7
    r = rng.random(n) * (a + b / 2.0)
    u = (-a + np.sqrt(a * a + 2.0 * b * r)) / b
    x = np.stack([np.clip(u * lx, 0.0, lx), rng.random(n) * ly, rng.random(n) * lz], axis=1)
    ma = (x[:, 1] < ly / 2).astype(np.float64)
    return W.Workload("ramp3s", p, x, np.stack([ma, 1.0 - ma, np.zeros(n)]), 3, {})


HOT_CASES = [
    ("rw2d", W.FP64), ("rw2d", W.FP32W_FP64ACC),
    ("rw3d", W.FP64), ("rw3d", W.FP32W_FP64ACC), ("rw3d", W.FP32_KAHAN),
    ("react3d", W.FP64), ("react3d", W.FP32W_FP64ACC),
    ("dense3d4", W.FP32W_FP64ACC), ("dense3d4", W.FP64), ("dense3d20", W.FP32W_FP64ACC),
    ("tens3d", W.FP32W_FP64ACC), ("plain2d", W.FP64),
    ("ramp3s", W.FP32W_FP64ACC), ("ramp3s", W.FP64),
]


@pytest.mark.parametrize("case,prec", HOT_CASES)
def test_hot_path_neighbor_sets(mt, oracle, case, prec):
    """Sec. 3, Eq. (1): the neighbour sets that the step's own passes use --
    the row-sum pass's candidates within the cutoff (trimmed rows in the
    3-d one-species workload), and the transfer pass's visited pairs (the
    row-sum pass's neighbour bits decoded over the same candidate rows and
    windows, or its own candidate loop for waves with more than 64
    candidates, and the global-memory path for tiles that do not fit the
    LDS) -- equal the oracle's K-D tree sets at the positions of that step,
    bit for bit."""
    if case == "rw2d":
        w = W.rw2d(n=40_000 + 13, steps=3, precision=prec)
    elif case == "rw3d":
        w = W.rw3d(n=30_000 + 19, steps=3, precision=prec, n_src=30)
    elif case == "react3d":
        w = W.react3d(n=40_000 + 21, steps=3, precision=prec)
    elif case == "dense3d4":
        w = _dense3d(30_000, 4.0, prec)      # rows of ~80: waves past 64 candidates
    elif case == "dense3d20":
        w = _dense3d(30_000, 20.0, prec)     # halos beyond the LDS: global path
    elif case == "ramp3s":
        w = _ramp3s(prec)
    elif case == "tens3d":
        w0 = W.rw3d(n=20_000 + 7, steps=3, precision=prec, n_src=20)
        w = W.Workload("tens3d", W.replace(w0.params, disp=W.rotated_tensor([2.5, 0.8, 0.5], [0.4, -0.3, 0.2])),
                       w0.x0, w0.m0, 3, {})
    else:
        w = W.plain2d(n=20_000, steps=3, precision=prec)
    steps = w.steps if case.startswith("dense") or case == "ramp3s" else 3
    say(f"  hot-path neighbours {case} {PREC_NAMES[prec]} n={w.params.n}")
    x, rs, tr = _hot_sets(mt, w, steps)
    ref = oracle_run(oracle, w, steps)
    assert np.array_equal(x, ref.x)
    orow, ocol = oracle.neighbors(ref.x, w.params.psi_eff, "kdtree", tens=oracle.tensor_of(w.params))
    for name, (row, col) in (("row-sum", rs), ("transfer", tr)):
        assert np.array_equal(row, orow), f"{name} pass: row lengths differ"
        assert np.array_equal(col, ocol), f"{name} pass: columns differ"


def test_neighbors_lattice_ties(mt, oracle):
    """Unit lattice with psi = 1 exactly: the r^2 = psi^2 ties are inside."""
    g = np.stack(np.meshgrid(np.arange(40.0), np.arange(30.0), indexing="xy"), -1).reshape(-1, 2)
    for psi in (1.0, np.nextafter(1.0, 0.0), 1.5):
        for prec in (W.FP64, W.FP32W_FP64ACC):
            p = W.Params(dim=2, n=len(g), lo=[0.0, 0.0, 0.0], hi=[39.0, 29.0, 0.0], d_rw=0.0,
                         d_mt=0.125, dt=1.0, beta=0.5, psi=float(psi), precision=prec)
            alloc = mt.TorchAllocator("cuda:0")
            with mt.Sim(p, g, np.ones((1, len(g))), allocator=alloc) as sim:
                row, col = sim.neighbors()
                sim.step(1)
                hot = [sim.step_neighbors(0), sim.step_neighbors(1)]
            orow, ocol = oracle.neighbors(g, float(psi), "brute")
            assert np.array_equal(row, orow) and np.array_equal(col, ocol)
            for hrow, hcol in hot:
                assert np.array_equal(hrow, orow) and np.array_equal(hcol, ocol)


# --------------------------------------------------- determinism / resume --
@pytest.mark.parametrize("prec", [W.FP64, W.FP32_KAHAN])
def test_deterministic_and_resume(mt, prec):
    w = W.rw2d(n=30_000, steps=6, precision=prec)
    a, xa, _ = gpu_run(mt, w, 6)
    b, xb, _ = gpu_run(mt, w, 6, chunks=[1, 2, 3])
    assert np.array_equal(a, b) and np.array_equal(xa, xb)
    h, xh, _ = gpu_run(mt, w, 3)
    p2 = W.Params(**{**w.params.as_dict(), "start_step": 3})
    w2 = W.Workload(w.name, p2, xh, h, 3)
    c, xc, _ = gpu_run(mt, w2, 3)
    assert np.array_equal(a, c) and np.array_equal(xa, xc)


@pytest.mark.parametrize("kind,prec", [("react3d", W.FP32W_FP64ACC), ("react3d", W.FP64),
                                       ("react3d", W.FP32_KAHAN), ("drift_tens3d", W.FP32W_FP64ACC)])
def test_resume_bitwise_variants(mt, kind, prec):
    """Three species with the reaction (whose masses the row-sum pass moves
    into the sorted order), and a drift with a rotated tensor: steps taken in
    chunks, or resumed at start_step from the exported state, equal one run."""
    if kind == "react3d":
        w = W.react3d(n=20_000 + 3, steps=6, precision=prec)
    else:
        w0 = W.rw3d(n=20_000 + 7, steps=6, precision=prec, n_src=20)
        w = W.Workload(kind, W.replace(w0.params, vel=[0.4, -0.2, 0.3],
                                       disp=W.rotated_tensor([2.0, 1.0, 0.5], [0.4, 0.1, 0.2])),
                       w0.x0, w0.m0, 6, {})
    a, xa, _ = gpu_run(mt, w, 6)
    b, xb, _ = gpu_run(mt, w, 6, chunks=[1, 2, 3])
    assert np.array_equal(a, b) and np.array_equal(xa, xb)
    h, xh, _ = gpu_run(mt, w, 3)
    p2 = W.Params(**{**w.params.as_dict(), "start_step": 3})
    c, xc, _ = gpu_run(mt, W.Workload(w.name, p2, xh, h, 3), 3)
    assert np.array_equal(a, c) and np.array_equal(xa, xc)


def test_static_resume_bitwise(mt):
    w = W.plain2d(n=5000, steps=10)
    a, _, _ = gpu_run(mt, w, 10)
    h, xh, _ = gpu_run(mt, w, 4)
    c, _, _ = gpu_run(mt, W.Workload(w.name, w.params, xh, h, 6), 6)
    assert np.array_equal(a, c)


@pytest.mark.parametrize("kind", ["rw2d", "plain2d"])
def test_stats_read_between_steps(mt, kind):
    """A step's totals and pair counters are completed either by the next
    step's first launch or, when something reads them first, on their own:
    reading them after every step gives the same counters, totals and masses
    as reading once after the same steps enqueued back to back."""
    w = W.rw2d(n=30_000, steps=5) if kind == "rw2d" else W.plain2d(n=5000, steps=5)
    alloc = mt.TorchAllocator("cuda:0")
    with mt.Sim(w.params, w.x0, w.m0, allocator=alloc) as sim:
        per = []
        for _ in range(5):
            sim.step(1)
            per.append(sim.stats())
        ma = sim.masses()
    with mt.Sim(w.params, w.x0, w.m0, allocator=alloc) as sim:
        sim.step(2)
        sim.step(3)
        mb = sim.masses()
        sb = sim.stats()
    sa = per[-1]
    assert np.array_equal(ma, mb)
    assert [p["steps_done"] for p in per] == [1, 2, 3, 4, 5]
    assert sa["steps_done"] == sb["steps_done"] == 5
    assert sa["pairs_total"] == sb["pairs_total"] and sa["pairs_last"] == sb["pairs_last"]
    assert sa["pairs_total"] == sum(p["pairs_last"] for p in per)
    assert np.array_equal(np.asarray(sa["mass_total"]), np.asarray(sb["mass_total"]))
    assert all(p["pairs_last"] > 0 for p in per)


# ------------------------------------------------------------ edge cases --
def test_edge_cases(mt, oracle):
    say("  edge: n=0")
    p = W.Params(dim=2, n=0, lo=[0, 0, 0], hi=[10, 10, 0], d_rw=0.5, d_mt=0.5, dt=0.1)
    with mt.Sim(p, np.zeros((0, 2)), np.zeros((1, 0)), allocator=mt.TorchAllocator()) as sim:
        sim.step(3)
        assert sim.masses().shape == (1, 0)
        assert sim.stats()["pairs_total"] == 0
    cases = []
    # one particle; a particle on every wall; everything inside one cell
    # (psi larger than the box); a ragged size just over a block and a tile
    cases.append(("one", W.Params(dim=3, n=1, lo=[0, 0, 0], hi=[5, 5, 5], d_rw=1.0, d_mt=1.0, dt=0.1,
                                  seed=5), np.array([[2.5, 2.5, 2.5]]), np.array([[1.0]])))
    xw = np.array([[0.0, 0.0], [10.0, 10.0], [0.0, 10.0], [10.0, 0.0], [5.0, 0.0], [0.3, 0.2]])
    cases.append(("walls", W.Params(dim=2, n=6, lo=[0, 0, 0], hi=[10, 10, 0], d_rw=0.0, d_mt=3.0, dt=1.0),
                  xw, np.arange(6.0)[None, :]))
    rng = np.random.default_rng(4)
    xs = rng.random((500, 2)) * 3.0
    cases.append(("one-cell", W.Params(dim=2, n=500, lo=[0, 0, 0], hi=[3, 3, 0], d_rw=0.2, d_mt=2.0,
                                       dt=0.5, seed=9), xs, rng.random((1, 500))))
    # 3000 particles in one cell: the tile overflows the LDS capacity of every
    # path, so both passes read their rows from global memory
    xc = rng.random((3000, 2)) * 2.0
    cases.append(("cluster", W.Params(dim=2, n=3000, lo=[0, 0, 0], hi=[2, 2, 0], d_rw=0.1, d_mt=2.0,
                                      dt=0.5, seed=13), xc, rng.random((1, 3000))))
    # ~20 particles per cell in 3-d: a plane's candidate rows hold more than
    # 64 particles, so the transfer pass takes the full candidate loop
    xd = rng.random((4320, 3)) * 6.0
    cases.append(("dense3d", W.Params(dim=3, n=4320, lo=[0, 0, 0], hi=[6, 6, 6], d_rw=0.05, d_mt=1.0 / 3.6,
                                      dt=0.1, seed=17), xd, rng.random((1, 4320))))
    xr = rng.random((4097 + 257, 3)) * [20, 7, 9]
    cases.append(("ragged", W.Params(dim=3, n=len(xr), lo=[0, 0, 0], hi=[20, 7, 9], d_rw=0.3, d_mt=0.6,
                                     dt=0.1, seed=11), xr, rng.random((1, len(xr)))))
    for name, p, x0, m0 in cases:
        for prec in (W.FP64, W.FP32W_FP64ACC):
            p.precision = prec
            say(f"  edge: {name} prec={PREC_NAMES[prec]}")
            w = W.Workload(name, p, x0, m0, 4)
            m, x, st = gpu_run(mt, w, 4)
            ref = oracle_run(oracle, w, 4, method="brute")
            assert np.array_equal(x, ref.x)
            assert normwise(m, ref.m) <= TOL[prec]
            assert st["pairs_total"] == int(ref.pairs.sum())


@pytest.mark.parametrize("prec", [W.FP64, W.FP32W_FP64ACC])
def test_dense_tile_global_histogram(mt, oracle, prec):
    """70000 particles inside the cells of one tile (a small psi in a large box
    makes the tiles 24 x 24 cells): the tile overflows the LDS, so both passes
    read its rows from global memory, and the transfer pass bins its
    particles through the global histogram, since the tile's LDS histogram
    holds 16-bit counts."""
    rng = np.random.default_rng(21)
    n = 70_000
    x0 = 0.2 + rng.random((n, 2)) * 4.1
    p = W.Params(dim=2, n=n, lo=[0, 0, 0], hi=[100, 100, 0], d_rw=0.001, d_mt=0.01, dt=0.1, seed=23,
                 precision=prec)
    w = W.Workload("dense-tile", p, x0, rng.random((1, n)), 3)
    m, x, st = gpu_run(mt, w, 3)
    ref = oracle_run(oracle, w, 3)
    assert np.array_equal(x, ref.x)
    assert normwise(m, ref.m) <= TOL[prec]
    assert st["pairs_total"] == int(ref.pairs.sum())


# --------------------------------------------------------------- full size --
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("prec", [W.FP64, W.FP32W_FP64ACC, W.FP32_KAHAN])
def test_advection_parity(mt, oracle, dim, prec):
    """Drift velocity (advection): positions bit for bit, masses at the bar.
    In 3-d the drift pushes particles against three walls within the run."""
    if dim == 2:
        w = W.adv2d(n=30_000 + 17, steps=6, precision=prec)
    else:
        w0 = W.rw3d(n=20_000 + 5, steps=6, precision=prec, n_src=20)
        w = W.Workload("adv3d", W.replace(w0.params, vel=[3.0, -2.0, 1.5]), w0.x0, w0.m0, 6, {})
    check_parity(mt, oracle, w, 6)
    # pure advection (no random walk): still re-binned every step
    p = W.replace(w.params, d_rw=0.0)
    check_parity(mt, oracle, W.Workload(w.name + "-pure", p, w.x0, w.m0, 6, {}), 6)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("prec", [W.FP64, W.FP32W_FP64ACC, W.FP32_KAHAN])
def test_tensor_parity(mt, oracle, dim, prec):
    """Dispersion tensor (Cholesky jumps, Mahalanobis kernel, ellipsoidal
    cutoff, all in the caller's frame): positions bit for bit, masses at the
    bar, neighbour sets bit-exact; a rotated tensor in 2-d, and in 3-d a
    rotated one with a drift and a diagonal one."""
    if dim == 2:
        w = W.aniso2d(n=30_000 + 29, steps=6, precision=prec)
        check_parity(mt, oracle, w, 6, nb=True)
    else:
        w0 = W.rw3d(n=20_000 + 7, steps=6, precision=prec, n_src=20)
        p = W.replace(w0.params, disp=W.rotated_tensor([2.5, 0.8, 0.5], [0.4, -0.3, 0.2]), vel=[1.0, 0.0, -2.0])
        check_parity(mt, oracle, W.Workload("tens3d", p, w0.x0, w0.m0, 6, {}), 6, nb=True)
        p = W.replace(w0.params, disp=W.diag_tensor([1.5, 0.8, 0.5]))
        check_parity(mt, oracle, W.Workload("diag3d", p, w0.x0, w0.m0, 6, {}), 6, nb=True)


@pytest.mark.parametrize("prec", [W.FP64, W.FP32W_FP64ACC])
def test_tensor_reaction_parity(mt, oracle, prec):
    """Three species with A+B->C under a dispersion tensor of determinant
    != 1: the reaction's concentrations use the box volume (the oracle
    computes them from the caller's box by definition)."""
    w0 = W.react3d(n=40_000 + 11, steps=4, precision=prec)
    p = W.replace(w0.params, disp=W.rotated_tensor([3.0, 1.5, 0.6], [0.5, 0.1, -0.2]))
    check_parity(mt, oracle, W.Workload("tens-react3d", p, w0.x0, w0.m0, 4, {}), 4)


@pytest.mark.parametrize("prec", [W.FP64, W.FP32W_FP64ACC])
def test_sparse_grid_many_scan_tiles(mt, oracle, prec):
    """3e6 particles with a tiny psi: the grid reaches its cap of ~4 cells
    per particle (over 2048 scan tiles, so the scan takes its top pass), the
    cells are smaller than a jump (most walked particles leave their tile and
    take the global-histogram slots), and a tile holds few particles."""
    n = 3_000_000
    L = math.sqrt(n)
    p = W.Params(dim=2, n=n, lo=[0.0, 0.0, 0.0], hi=[L, L, 0.0], d_rw=0.5, d_mt=0.002, dt=0.1,
                 beta=0.5, psi=0.0, seed=0x4D54505409, precision=prec)
    x = W._uniform(20220409, n, 2, p.lo, p.hi)
    m = np.random.default_rng(9).random((1, n))
    w = W.Workload("sparse2d", p, x, m, 3, {})
    m_, x_, st, ref = check_parity(mt, oracle, w, 3)
    assert st["n_cells"] + 1 > 2048 * 4096
