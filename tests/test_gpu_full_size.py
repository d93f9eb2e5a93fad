"""Parity at the full sizes of the three large workloads, in the launch
configuration the benchmark times (one sim, the library's own tiles):
the first steps against the CPU oracle element by element, then invariants
over longer runs.  Collected first among the GPU tests."""
import numpy as np
import pytest

from paper_2204_03756_amd import workloads as W

from gpu_helpers import check_parity, gpu_run, load_mt, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mt():
    return load_mt()


def test_rw3d_full_size_first_step(mt, oracle):
    """2e6 particles, 3-d: the first step against the oracle in FP64 and
    FP32W (masses element by element at the bar, positions bit for bit, pair
    counts exact), then 100 Kahan steps of invariants."""
    for prec in (W.FP64, W.FP32W_FP64ACC):
        check_parity(mt, oracle, W.rw3d(precision=prec), 1)
    w = W.rw3d(precision=W.FP32_KAHAN)
    m, x, st = gpu_run(mt, w, 100)
    assert st["nonfinite"] == 0 and st["drift"] < 1e-4
    assert m.min() >= -1e-9
    say(f"  rw3d kahan 100 steps: drift {st['drift']:.3e}")


@pytest.mark.parametrize("prec", [W.FP32W_FP64ACC, W.FP64])
def test_react3d_full_size_parity(mt, oracle, prec):
    """3.2e7 particles, three species, A+B->C (the largest workload, in the
    launch configuration the benchmark times): the first step against the
    oracle -- masses of all three species element by element at the bar
    (Sec. 3, Eq. (5), then the reaction), positions bit for bit, the pair
    count exact, the device totals at the bar."""
    w = W.react3d(precision=prec)
    check_parity(mt, oracle, w, 1)


def test_react3d_full_size_invariants(mt):
    """3.2e7 particles, the workload's 200 steps: the transfer conserves
    A + C and B + C, the reaction makes C, no mass goes negative, every
    particle stays in the box, and the pair count stays that of the
    uniform density."""
    w = W.react3d(precision=W.FP32W_FP64ACC)
    m, x, st = gpu_run(mt, w, w.steps)
    assert st["nonfinite"] == 0 and st["steps_done"] == w.steps
    ta, tb = m[0].sum() + m[2].sum(), m[1].sum() + m[2].sum()
    assert abs(ta / w.m0[0].sum() - 1) < 1e-9 and abs(tb / w.m0[1].sum() - 1) < 1e-9
    assert m[2].sum() > 0 and m.min() > -1e-12
    assert np.all((x >= 0) & (x <= w.params.hi[0]))
    # ordered pairs per particle: (4/3) pi psi^3 at density 1 (5.92), less
    # the walls' share; a walk that lost uniformity would move it
    per = st["pairs_last"] / w.params.n
    assert 5.7 < per < 5.95, per
    say(f"  react3d {w.steps} steps: C total {m[2].sum():.6e}, pairs/particle {per:.4f}")


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


def test_long_runs_keep_the_invariants(mt):
    """Thousands of steps (far past the workloads' 50-200): the walking 2-d
    sim and the static one conserve their mass to roundoff, keep the maximum
    principle of beta = 1/2 (no mass leaves [0, max m0]), keep every particle
    in the box, and the walking sim keeps the pair count of its uniform
    density; the step counters add up."""
    for w, steps in ((W.rw2d(n=400_000, precision=W.FP32W_FP64ACC), 4000),
                     (W.plain2d(n=10_000, precision=W.FP64), 5000)):
        m, x, st = gpu_run(mt, w, steps)
        assert st["nonfinite"] == 0 and st["steps_done"] == steps
        assert st["drift"] < 1e-11, st["drift"]
        assert m.min() >= -1e-15 and m.max() <= w.m0.max() * (1 + 1e-12)
        assert np.all((x >= 0) & (x <= w.params.hi[0]))
        per = st["pairs_last"] / w.params.n
        say(f"  {w.name} {steps} steps: drift {st['drift']:.3e}, pairs/particle {per:.3f}, "
            f"pairs total {st['pairs_total']}")
        if w.params.d_rw > 0:
            # pi psi^2 at density 1 (5.65), less the walls' share
            assert 5.4 < per < 5.70, per
        assert st["pairs_total"] >= st["pairs_last"] * steps * 0.98
