"""Serving pool on the GPU: continuous batching of independent sims.

* Every result out of the pool equals the same sim run alone, bit for bit,
  and the oracle within the FP32 bar.
* Requests arriving while others run are admitted as slots and budget free
  up; admission beyond the budget or the slots is refused (retry later).
"""
import numpy as np
import pytest

from paper_2204_03756_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2204_03756_amd import mtpt
    mtpt.load()
    return mtpt


def alone(mt, r):
    with mt.Sim(r.params, r.x0, r.m0, allocator=mt.TorchAllocator()) as sim:
        sim.step(r.steps)
        return sim.masses()


def test_pool_alone_equals_mix(mt, oracle):
    reqs = [W.request(i, n_min=2e3, n_max=3e4) for i in range(10)]
    for r in reqs:
        r.steps = min(r.steps, 25)
    pool = mt.mtpt_pool_create(0, 4)
    try:
        pending = list(reqs)
        active = {}
        results = {}
        ticks = 0
        while pending or active:
            # admit while slots free up (continuous batching)
            while pending:
                r = pending[0]
                t = mt.mtpt_pool_admit(pool, r.params, r.x0, r.m0, r.steps)
                if t is None:
                    break
                active[t] = r
                pending.pop(0)
            assert len(active) <= 4
            mt.mtpt_pool_tick(pool)
            ticks += 1
            for t in list(active):
                if mt.mtpt_pool_done(pool, t):
                    r = active.pop(t)
                    results[r.rid] = mt.mtpt_pool_result(pool, t, r.params.n, 1)
        print(f"  pool: {len(reqs)} sims in {ticks} ticks", flush=True)
    finally:
        mt.mtpt_pool_destroy(pool)
    for r in reqs:
        a = alone(mt, r)
        assert np.array_equal(a, results[r.rid]), f"request {r.rid} differs alone vs in the mix"
    for r in reqs[:4]:
        ref = oracle.run(r.params, r.x0, r.m0, r.steps)
        err = np.max(np.abs(results[r.rid] - ref.m)) / np.max(np.abs(ref.m))
        assert err <= 1e-5


def test_pool_large_requests_match_the_oracle(mt, oracle):
    """Two large requests of the serving mix's shape -- a 2-d sim of ~1e6
    particles and a 3-d one of ~3e5, 100 and 120 steps, Kahan FP32 -- run
    together in the pool with small requests admitted around them: the
    large results equal the oracle within the FP32 bar, and the small ones
    equal their solo runs bit for bit."""
    big = [W.request(101, n_min=9.0e5, n_max=1.0e6), W.request(102, n_min=2.9e5, n_max=3.0e5)]
    big[0].steps, big[1].steps = 100, 120
    small = [W.request(200 + i, n_min=1e4, n_max=3e4) for i in range(6)]
    for r in small:
        r.steps = min(r.steps, 40)
    say = lambda *a: print(*a, flush=True)
    say(f"  pool: large dims {[r.params.dim for r in big]} n {[r.params.n for r in big]}")
    pool = mt.mtpt_pool_create(0, 4)
    results = {}
    try:
        pending = big + small
        active = {}
        ticks = 0
        while pending or active:
            while pending:
                r = pending[0]
                t = mt.mtpt_pool_admit(pool, r.params, r.x0, r.m0, r.steps)
                if t is None:
                    break
                active[t] = r
                pending.pop(0)
            mt.mtpt_pool_tick(pool)
            ticks += 1
            for t in list(active):
                if mt.mtpt_pool_done(pool, t):
                    r = active.pop(t)
                    results[r.rid] = mt.mtpt_pool_result(pool, t, r.params.n, 1)
        say(f"  pool: {len(results)} sims in {ticks} ticks")
    finally:
        mt.mtpt_pool_destroy(pool)
    for r in big:
        ref = oracle.run(r.params, r.x0, r.m0, r.steps)
        err = np.max(np.abs(results[r.rid] - ref.m)) / np.max(np.abs(ref.m))
        say(f"  pool large request {r.rid}: normwise {err:.3e}")
        assert err <= 1e-5
    for r in small:
        assert np.array_equal(alone(mt, r), results[r.rid])


def test_sim_bytes_equal_the_allocation(mt):
    """mtpt_sim_bytes (the admission estimate) equals what create allocates,
    also with a rotated dispersion tensor (cells stretched per axis)."""
    class Counting(mt.TorchAllocator):
        def __init__(self):
            super().__init__("cuda:0")
            self.sizes = []

        def _alloc(self, nbytes, ctx):
            self.sizes.append(int(nbytes))
            return super()._alloc(nbytes, ctx)
    for w in (W.rw2d(n=50_000), W.aniso2d(n=50_000),
              W.Workload("t3", W.replace(W.react3d(n=60_000).params,
                                         disp=W.rotated_tensor([3.0, 1.0, 0.5], [0.3, 0.2, 0.1])),
                         W.react3d(n=60_000).x0, W.react3d(n=60_000).m0, 1, {})):
        alloc = Counting()
        sim = mt.Sim(w.params, w.x0, w.m0, allocator=alloc)
        sim.close()
        assert alloc.sizes[0] == mt.mtpt_sim_bytes(w.params), w.name


def test_pool_admission_budget_and_slots(mt):
    r = W.request(3, n_min=5e3, n_max=6e3)
    need = mt.mtpt_sim_bytes(r.params)
    pool = mt.mtpt_pool_create(int(need * 1.5 + r.params.n * 8), 8)
    try:
        t1 = mt.mtpt_pool_admit(pool, r.params, r.x0, r.m0, 3)
        assert t1 is not None
        assert mt.mtpt_pool_admit(pool, r.params, r.x0, r.m0, 3) is None   # over budget
        active, held, budget = mt.mtpt_pool_usage(pool)
        assert active == 1 and held <= budget
        with pytest.raises(mt.MtptError):
            mt.mtpt_pool_result(pool, t1, r.params.n, 1)                   # not finished
        while not mt.mtpt_pool_done(pool, t1):
            mt.mtpt_pool_tick(pool)
        mt.mtpt_pool_result(pool, t1, r.params.n, 1)
        assert mt.mtpt_pool_admit(pool, r.params, r.x0, r.m0, 3) is not None
    finally:
        mt.mtpt_pool_destroy(pool)
    pool = mt.mtpt_pool_create(0, 1)
    try:
        assert mt.mtpt_pool_admit(pool, r.params, r.x0, r.m0, 2) is not None
        assert mt.mtpt_pool_admit(pool, r.params, r.x0, r.m0, 2) is None   # no slot
    finally:
        mt.mtpt_pool_destroy(pool)


def test_pool_batches_every_kernel_variant(mt, oracle):
    """One pool holding a sim of every kind it batches separately -- static
    and moving, 2-d and 3-d, the three precisions, one and three species
    (with the reaction), a drift, dispersion tensors -- so that each group's
    batched kernels run beside the others': every result equals the same sim
    run alone bit for bit, and the oracle within its precision's bar."""
    from gpu_helpers import TOL, normwise
    t3 = W.rotated_tensor([3.0, 1.0, 0.5], [0.3, 0.2, 0.1])
    r3 = W.react3d(n=20_000 + 3, steps=5, precision=W.FP32W_FP64ACC)
    d3 = W.rw3d(n=15_000 + 9, steps=5, precision=W.FP64, n_src=20)
    ws = [
        W.plain2d(n=5000, steps=6, precision=W.FP64),
        W.plain2d(n=7000, steps=6, precision=W.FP32W_FP64ACC),
        r3,
        W.react3d(n=12_000 + 1, steps=4, precision=W.FP64),
        W.react3d(n=12_000 + 5, steps=4, precision=W.FP32_KAHAN),
        W.aniso2d(n=20_000 + 7, steps=5, precision=W.FP32_KAHAN),
        W.adv2d(n=20_000 + 11, steps=5, precision=W.FP32W_FP64ACC),
        W.Workload("drift3d", W.replace(d3.params, vel=[0.5, -0.3, 0.2]), d3.x0, d3.m0, 5, {}),
        W.Workload("tens_react3d", W.replace(r3.params, disp=t3, seed=0x4D54505477), r3.x0, r3.m0, 4, {}),
    ]
    reqs = [W.Request(900 + i, 0.0, w.params, w.x0, w.m0, w.steps) for i, w in enumerate(ws)]
    pool = mt.mtpt_pool_create(0, len(reqs))
    results = {}
    try:
        active = {}
        for r in reqs:
            t = mt.mtpt_pool_admit(pool, r.params, r.x0, r.m0, r.steps)
            assert t is not None
            active[t] = r
        while active:
            mt.mtpt_pool_tick(pool)
            for t in list(active):
                if mt.mtpt_pool_done(pool, t):
                    r = active.pop(t)
                    results[r.rid] = mt.mtpt_pool_result(pool, t, r.params.n, r.params.n_species)
    finally:
        mt.mtpt_pool_destroy(pool)
    for w, r in zip(ws, reqs):
        a = alone(mt, r)
        assert np.array_equal(a, results[r.rid]), f"{w.name} differs alone vs in the mix"
        ref = oracle.run(r.params, r.x0, r.m0, r.steps)
        err = normwise(results[r.rid], ref.m)
        print(f"  pool variant {w.name} prec {r.params.precision}: normwise {err:.3e}", flush=True)
        assert err <= TOL[r.params.precision], w.name
