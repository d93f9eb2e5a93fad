"""Randomised parity: small sims drawn over the parameter space the C-ABI
accepts -- dimension, precision, one or three species (with and without the
reaction), static or walking particles, a drift, a rotated dispersion tensor,
beta, an explicit or default psi, boxes off the origin of uneven sides and
densities from sparse to dense -- each against the oracle at its precision's
bar, positions bit for bit and pair counts exact.  The draws are seeded, so
every run checks the same cases."""
import math

import numpy as np
import pytest

from paper_2204_03756_amd import workloads as W

pytestmark = pytest.mark.gpu

from gpu_helpers import PREC_NAMES, check_parity, load_mt, say  # noqa: E402

N_CASES = 80


@pytest.fixture(scope="module")
def mt():
    return load_mt()


def draw_case(k: int) -> W.Workload:
    rng = np.random.Generator(np.random.Philox(0x5EED0000 + k))
    dim = int(rng.integers(2, 4))
    prec = int(rng.integers(0, 3))
    ns = 3 if rng.random() < 0.35 else 1
    d_mt = float(rng.uniform(0.1, 2.0))
    dt = float(rng.uniform(0.02, 0.2))
    d_rw = 0.0 if rng.random() < 0.2 else float(rng.uniform(0.05, 1.5))
    beta = float(rng.choice([0.25, 0.5, 1.0]))
    psi_def = 3.0 * math.sqrt(4.0 * d_mt * dt)
    psi = 0.0 if rng.random() < 0.6 else float(psi_def * rng.uniform(0.5, 1.5))
    lo = [float(v) for v in rng.uniform(-20.0, 20.0, 3)]
    sides = rng.uniform(4.0, 30.0, 3) * (psi if psi > 0 else psi_def)
    hi = [lo[i] + float(sides[i]) for i in range(3)]
    if dim == 2:
        lo[2], hi[2] = 0.0, 0.0
    vol = float(np.prod(sides[:dim]))
    dens_per_cell = float(rng.choice([0.3, 1.5, 6.0, 20.0]))
    cell_vol = (psi if psi > 0 else psi_def) ** dim
    n = int(np.clip(dens_per_cell * vol / cell_vol, 50, 20000))
    vel = [0.0, 0.0, 0.0]
    if rng.random() < 0.3:
        vel = [float(v) for v in rng.uniform(-1.0, 1.0, 3)]
        if dim == 2:
            vel[2] = 0.0
    disp = [0.0] * 9
    if rng.random() < 0.3:
        eigs = rng.uniform(0.4, 3.0, dim).tolist()
        ang = rng.uniform(0.0, math.pi, 1 if dim == 2 else 3).tolist()
        disp = W.rotated_tensor(eigs, ang)
    k_react = float(rng.choice([0.0, 0.5, 2.0])) if ns == 3 else 0.0
    p = W.Params(dim=dim, n=n, lo=lo, hi=hi, d_rw=d_rw, d_mt=d_mt, dt=dt, beta=beta, psi=psi,
                 k_react=k_react, n_species=ns, seed=0x4D545054A000 + k, precision=prec,
                 vel=vel, disp=disp)
    u = rng.random((n, dim))
    x = np.minimum(np.asarray(lo[:dim]) + u * np.asarray(sides[:dim]), np.asarray(hi[:dim]))
    m = rng.uniform(0.0, 1.0, (ns, n))
    steps = int(rng.integers(1, 7))
    return W.Workload(f"random{k}", p, x, m, steps, {})


@pytest.mark.parametrize("k", range(N_CASES))
def test_random_config_parity(mt, oracle, k):
    w = draw_case(k)
    p = w.params
    say(f"  case {k}: d={p.dim} {PREC_NAMES[p.precision]} S={p.n_species} k={p.k_react} n={p.n} "
        f"d_rw={p.d_rw:.3g} beta={p.beta} psi={p.psi:.3g} drift={any(v != 0 for v in p.vel)} "
        f"tensor={any(v != 0 for v in p.disp)} steps={w.steps}")
    check_parity(mt, oracle, w, w.steps)


def test_random_configs_in_one_pool(mt):
    """Twenty of the draws admitted together into one pool (their kernels
    batched by kind, their steps interleaved): every result equals the same
    sim run alone, bit for bit."""
    ws = [draw_case(k) for k in range(20)]
    pool = mt.mtpt_pool_create(0, len(ws))
    results = {}
    try:
        active = {}
        for i, w in enumerate(ws):
            t = mt.mtpt_pool_admit(pool, w.params, w.x0, w.m0, w.steps)
            assert t is not None
            active[t] = i
        while active:
            mt.mtpt_pool_tick(pool)
            for t in list(active):
                if mt.mtpt_pool_done(pool, t):
                    i = active.pop(t)
                    results[i] = mt.mtpt_pool_result(pool, t, ws[i].params.n, ws[i].params.n_species)
    finally:
        mt.mtpt_pool_destroy(pool)
    alloc = mt.TorchAllocator("cuda:0")
    for i, w in enumerate(ws):
        with mt.Sim(w.params, w.x0, w.m0, allocator=alloc) as sim:
            sim.step(w.steps)
            a = sim.masses()
        assert np.array_equal(a, results[i]), f"draw {i} differs alone vs in the pool"


@pytest.mark.parametrize("k", range(0, N_CASES, 4))
def test_random_config_hot_neighbor_sets(mt, oracle, k):
    """Sec. 3, Eq. (1): on every fourth draw, the pairs the last step's
    row-sum and transfer passes used equal the oracle's K-D tree sets at the
    positions of that step, bit for bit."""
    w = draw_case(k)
    alloc = mt.TorchAllocator("cuda:0")
    with mt.Sim(w.params, w.x0, w.m0, allocator=alloc) as sim:
        sim.step(w.steps)
        x = sim.positions()
        hot = (sim.step_neighbors(0), sim.step_neighbors(1))
    ref = oracle.run(w.params, w.x0, w.m0, w.steps)
    assert np.array_equal(x, ref.x)
    orow, ocol = oracle.neighbors(ref.x, w.params.psi_eff, "kdtree", tens=oracle.tensor_of(w.params))
    for name, (row, col) in zip(("row-sum", "transfer"), hot):
        assert np.array_equal(row, orow), f"draw {k}, {name} pass: row lengths differ"
        assert np.array_equal(col, ocol), f"draw {k}, {name} pass: columns differ"
