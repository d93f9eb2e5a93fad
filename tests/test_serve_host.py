"""Host-side tests of the serving loop against a fake device (no GPU):
admission by slots and budget, FIFO order, continuous batching (late arrivals
join while others run), rejection of requests that can never fit, isolation
of a failed admission."""
import numpy as np

from paper_2204_03756_amd import serve, workloads as W


class Tracking(serve.FakeBackend):
    def __init__(self, *a, **k):
        super().__init__(*a, **k)
        self.max_active = 0
        self.max_held = 0
        self.admit_order = []

    def admit(self, params, x0, m0, steps):
        t = super().admit(params, x0, m0, steps)
        if t is not None:
            self.admit_order.append(int(params.n))
        self.max_active = max(self.max_active, len(self.active))
        self.max_held = max(self.max_held, self.held)
        return t


def _reqs(sizes, steps):
    out = []
    for k, (n, st) in enumerate(zip(sizes, steps)):
        p = W.Params(dim=2, n=n, lo=[0, 0, 0], hi=[10, 10, 0], d_rw=0.5, d_mt=0.5, dt=0.1)
        out.append(W.Request(k, 0.0, p, np.zeros((n, 2)), np.zeros((1, n)), st))
    return out


def test_slots_and_budget_are_respected():
    reqs = _reqs([1000] * 12, [5, 9, 3, 7] * 3)
    be = Tracking(budget=4 * (1000 * 100 + 4096), max_slots=3)
    rep = serve.serve(be, reqs, realtime=False)
    assert len(rep.outcomes) == 12 and not rep.rejected
    assert be.max_active <= 3 and be.max_held <= be.budget
    assert all(o.latency >= 0 and o.finished >= o.admitted for o in rep.outcomes.values())


def test_continuous_batching_admits_late_arrivals_while_others_run():
    reqs = _reqs([500, 500, 500], [50, 50, 5])
    arrivals = [0.0, 0.0, 0.0]
    be = Tracking(budget=10**9, max_slots=2)
    rep = serve.serve(be, reqs, arrivals, realtime=False)
    o = rep.outcomes
    # the short third request waits for a slot, and finishes before the two long ones would
    # have finished had it been queued behind both
    assert o[2].admitted >= min(o[0].finished, o[1].finished) or rep.ticks >= 50
    assert rep.ticks < 50 + 50 + 5


def test_fifo_and_rejection():
    reqs = _reqs([300, 10_000_000, 200, 100], [3, 3, 3, 3])
    be = Tracking(budget=10**6, max_slots=8)
    rep = serve.serve(be, reqs, realtime=False)
    assert rep.rejected == [1]
    assert be.admit_order == [300, 200, 100]
    assert sorted(rep.outcomes) == [0, 2, 3]


def test_failed_admission_is_isolated():
    reqs = _reqs([100, 777, 300], [2, 2, 2])
    be = Tracking(budget=10**8, max_slots=8, fail_admit=[777])
    rep = serve.serve(be, reqs, realtime=False)
    assert rep.rejected == [1] and sorted(rep.outcomes) == [0, 2]


def test_poisson_arrivals_replay():
    reqs = [W.request(i, n_min=1e3, n_max=3e3) for i in range(20)]
    arr = W.arrivals(20, rate=50.0)
    assert np.all(np.diff(arr) >= 0) and arr[0] > 0
    be = Tracking(budget=10**9, max_slots=4)
    rep = serve.serve(be, reqs, arr, realtime=False)
    s = rep.summary()
    assert s["sims"] == 20 and s["p99_latency_s"] >= s["p50_latency_s"] >= 0
