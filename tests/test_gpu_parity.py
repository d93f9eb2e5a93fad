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

TOL = {W.FP64: 1e-12, W.FP32W_FP64ACC: 1e-5, W.FP32_KAHAN: 1e-5}
PREC_NAMES = {W.FP64: "fp64", W.FP32W_FP64ACC: "fp32w", W.FP32_KAHAN: "kahan"}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2204_03756_amd import mtpt
    mtpt.load()
    return mtpt


def normwise(m, ref):
    out = []
    for c in range(ref.shape[0]):
        den = np.max(np.abs(ref[c]))
        out.append(float(np.max(np.abs(m[c] - ref[c])) / den) if den > 0 else float(np.max(np.abs(m[c]))))
    return max(out)


def gpu_run(mt, w, steps, chunks=None):
    say(f"  gpu: {w.name} n={w.params.n} prec={PREC_NAMES[w.params.precision]} steps={steps}")
    alloc = mt.TorchAllocator("cuda:0")
    with mt.Sim(w.params, w.x0, w.m0, allocator=alloc) as sim:
        for k in (chunks or [steps]):
            sim.step(k)
        return sim.masses(), sim.positions(), sim.stats()


def oracle_run(oracle, w, steps, **kw):
    return oracle.run(w.params, w.x0, w.m0, steps, **kw)


def check_parity(mt, oracle, w, steps, bitwise_pos=True):
    m, x, st = gpu_run(mt, w, steps)
    ref = oracle_run(oracle, w, steps)
    err = normwise(m, ref.m)
    say(f"  {w.name} {PREC_NAMES[w.params.precision]}: normwise {err:.3e}, drift {st['drift']:.3e}, "
        f"pairs/step {st['pairs_last']}")
    assert err <= TOL[w.params.precision]
    if bitwise_pos:
        assert np.array_equal(x, ref.x)
    assert st["pairs_last"] == int(ref.pairs[-1])
    assert st["pairs_total"] == int(ref.pairs.sum())
    assert st["steps_done"] == steps
    for c in range(ref.m.shape[0]):
        # the device's FP64 totals against the oracle's compensated totals,
        # at the path's bar
        assert abs(st["mass_total"][c] - ref.totals[-1, c]) <= \
            TOL[w.params.precision] * max(1.0, abs(ref.totals[-1, c]))
    return m, x, st, ref


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
            orow, ocol = oracle.neighbors(g, float(psi), "brute")
            assert np.array_equal(row, orow) and np.array_equal(col, ocol)


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
def test_rw2d_full_size_first_steps(mt, oracle):
    """4e6 particles: the first two steps against the oracle, then 100 steps
    of invariants (conservation, maximum principle for beta = 1/2)."""
    for prec in (W.FP32W_FP64ACC, W.FP64):
        w = W.rw2d(precision=prec)
        check_parity(mt, oracle, w, 2)
    w = W.rw2d(precision=W.FP32W_FP64ACC)
    m, x, st = gpu_run(mt, w, 100)
    assert st["nonfinite"] == 0
    assert st["drift"] < 1e-12
    assert m.min() >= -1e-15 and m.max() <= w.m0.max() * (1 + 1e-12)
    assert np.all((x >= 0) & (x <= w.params.hi[0]))
    say(f"  rw2d 100 steps: drift {st['drift']:.3e}, pairs/step {st['pairs_last']}")


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
def test_anisotropic_parity(mt, oracle, dim, prec):
    """Diagonal dispersion tensor (the isotropic step in the scaled frame):
    positions bit for bit in the caller's frame, masses at the bar; in 3-d
    with a drift as well."""
    if dim == 2:
        w = W.aniso2d(n=30_000 + 29, steps=6, precision=prec)
    else:
        w0 = W.rw3d(n=20_000 + 7, steps=6, precision=prec, n_src=20)
        p = W.replace(w0.params, aniso=[1.5, 0.8, 0.5], vel=[1.0, 0.0, -2.0])
        w = W.Workload("aniso3d", p, w0.x0, w0.m0, 6, {})
    check_parity(mt, oracle, w, 6)


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


def test_rw3d_full_size_first_step(mt, oracle):
    w = W.rw3d(precision=W.FP32W_FP64ACC)
    check_parity(mt, oracle, w, 1)
    w = W.rw3d(precision=W.FP32_KAHAN)
    m, x, st = gpu_run(mt, w, 100)
    assert st["nonfinite"] == 0 and st["drift"] < 1e-4
    assert m.min() >= -1e-9
    say(f"  rw3d kahan 100 steps: drift {st['drift']:.3e}")


def test_react3d_full_size_invariants(mt, oracle):
    """3.2e7 particles, three species: positions of sampled pids against the
    oracle's walk after one step, and the reaction/transfer invariants after
    20 steps."""
    w = W.react3d(precision=W.FP32W_FP64ACC)
    m, x, st = gpu_run(mt, w, 1)
    rng = np.random.default_rng(0)
    sample = rng.choice(w.params.n, 2000, replace=False)
    x32 = w.x0[sample].astype(np.float32).astype(np.float64)
    # the oracle's normals of the sampled pids, walked in float as the FP32
    # state requires
    for k, pid in enumerate(sample[:200]):
        z0, z1 = oracle.normal_pair(w.params.seed, 0, int(pid), 0)
        z2, _ = oracle.normal_pair(w.params.seed, 0, int(pid), 1)
        exp = []
        for d, z in enumerate((z0, z1, z2)):
            v = np.float32(x32[k, d]) + np.float32(z * math.sqrt(2.0 * w.params.d_rw * w.params.dt))
            lo, hi = np.float32(0.0), np.float32(w.params.hi[d])
            while v < lo or v > hi:
                v = np.float32(2.0) * lo - v if v < lo else np.float32(2.0) * hi - v
            exp.append(float(v))
        assert np.array_equal(x[pid], exp)
    m, x, st = gpu_run(mt, w, 20)
    assert st["nonfinite"] == 0
    ta, tb = m[0].sum() + m[2].sum(), m[1].sum() + m[2].sum()
    assert abs(ta / w.m0[0].sum() - 1) < 1e-9 and abs(tb / w.m0[1].sum() - 1) < 1e-9
    assert m[2].sum() > 0 and m.min() > -1e-12
    say(f"  react3d 20 steps: C total {m[2].sum():.6e}")
