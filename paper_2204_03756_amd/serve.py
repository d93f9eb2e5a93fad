"""Serving loop: continuous batching of independent MTPT simulations.

Requests (independent sims of any size and dimension) arrive over time.  The
loop admits every arrived request that the pool can hold now (slots and
device-memory budget), advances all admitted sims together -- one batched
launch per phase per tick, so sims admitted at different times overlap on the
device -- collects each sim the tick its last step is enqueued, and frees its
slot for the requests waiting behind it.  Request latency is the time from
arrival to the result being on the host.

The loop talks to a backend with the pool's interface.  ``PoolBackend`` is the
C-ABI pool of libmtpt.so (all arithmetic on the GPU); ``FakeBackend`` is a
host-only model of slots, memory and step counts, used to test the scheduling
logic without a GPU.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np


@dataclass
class Outcome:
    rid: int
    arrival: float
    admitted: float
    finished: float
    masses: Optional[np.ndarray]
    pairs_total: int = 0

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class Report:
    outcomes: Dict[int, Outcome]
    wall_s: float
    ticks: int
    rejected: List[int] = field(default_factory=list)

    def latencies(self) -> np.ndarray:
        return np.array(sorted(o.latency for o in self.outcomes.values()))

    def summary(self) -> dict:
        lat = self.latencies()
        pairs = sum(o.pairs_total for o in self.outcomes.values())
        pct = (lambda q: float(lat[min(len(lat) - 1, max(0, int(math.ceil(q * len(lat))) - 1))])
               if len(lat) else float("nan"))
        return {
            "sims": len(self.outcomes), "wall_s": self.wall_s,
            "sims_per_s": len(self.outcomes) / self.wall_s if self.wall_s > 0 else float("nan"),
            "p50_latency_s": pct(0.50), "p99_latency_s": pct(0.99),
            "pair_updates_per_s": pairs / self.wall_s if self.wall_s > 0 else float("nan"),
            "ticks": self.ticks, "rejected": len(self.rejected),
        }


class PoolBackend:
    """The GPU pool of libmtpt.so."""

    def __init__(self, hbm_budget: int = 0, max_slots: int = 64, allocator=None, stream=None):
        from . import mtpt
        self._m = mtpt
        self.pool = mtpt.mtpt_pool_create(hbm_budget, max_slots, stream, allocator)

    def sim_bytes(self, params) -> int:
        return self._m.mtpt_sim_bytes(params)

    def admit(self, params, x0, m0, steps) -> Optional[int]:
        return self._m.mtpt_pool_admit(self.pool, params, x0, m0, steps)

    def tick(self) -> int:
        return self._m.mtpt_pool_tick(self.pool)

    def done(self, ticket: int) -> bool:
        return self._m.mtpt_pool_done(self.pool, ticket)

    def result(self, ticket: int, n: int, ns: int):
        st = self._m.mtpt_pool_stats(self.pool, ticket)
        m = self._m.mtpt_pool_result(self.pool, ticket, n, ns)
        return m, int(st["pairs_total"])

    def usage(self):
        return self._m.mtpt_pool_usage(self.pool)

    def close(self):
        if self.pool is not None:
            self._m.mtpt_pool_destroy(self.pool)
            self.pool = None


class FakeBackend:
    """Host-only model of the pool: a byte budget, a slot limit, and sims that
    finish after their number of ticks.  ``bytes_per_particle`` stands in for
    the library's buffer plan; ``fail_admit`` lists request sizes whose
    admission raises (an injected device failure)."""

    def __init__(self, budget: int, max_slots: int, bytes_per_particle: int = 100,
                 fail_admit=()):
        self.budget = budget
        self.max_slots = max_slots
        self.bpp = bytes_per_particle
        self.fail_admit = set(fail_admit)
        self.active = {}          # ticket -> [steps_done, steps_target, bytes]
        self.held = 0
        self.next = 1

    def sim_bytes(self, params) -> int:
        return int(params.n) * self.bpp + 4096

    def admit(self, params, x0, m0, steps) -> Optional[int]:
        if int(params.n) in self.fail_admit:
            raise RuntimeError("injected admission failure")
        need = self.sim_bytes(params)
        if len(self.active) >= self.max_slots or self.held + need > self.budget:
            return None
        t = self.next
        self.next += 1
        self.active[t] = [0, int(steps), need]
        self.held += need
        return t

    def tick(self) -> int:
        done = 0
        for st in self.active.values():
            if st[0] < st[1]:
                st[0] += 1
                done += st[0] == st[1]
        return done

    def done(self, ticket: int) -> bool:
        st = self.active[ticket]
        return st[0] >= st[1]

    def result(self, ticket: int, n: int, ns: int):
        st = self.active.pop(ticket)
        if st[0] < st[1]:
            raise RuntimeError("not finished")
        self.held -= st[2]
        return None, 0

    def usage(self):
        return len(self.active), self.held, self.budget

    def close(self):
        self.active.clear()


def serve(backend, requests, arrivals=None, realtime: bool = True, max_wait_s: float = 600.0,
          clock=time.perf_counter, sleep=time.sleep) -> Report:
    """Run the request loop until every request is answered (or rejected).

    requests  list of workloads.Request (params, x0, m0, steps)
    arrivals  arrival times in seconds after the start (default: all at 0)
    realtime  wait for arrivals in real time; otherwise time jumps to the
              next arrival when the pool is idle (a replay).
    A request whose sim can never fit (larger than the whole budget) is
    rejected, not queued forever."""
    if arrivals is None:
        arrivals = [0.0] * len(requests)
    order = sorted(range(len(requests)), key=lambda k: (arrivals[k], requests[k].rid))
    pending = collections.deque(order)
    waiting = collections.deque()
    active = {}                    # ticket -> (request index, admitted time)
    outcomes: Dict[int, Outcome] = {}
    rejected = []
    ticks = 0
    _, _, budget = backend.usage()
    t0 = clock()
    offset = 0.0                   # replay mode: skipped idle time

    def now():
        return clock() - t0 + offset

    while pending or waiting or active:
        t = now()
        while pending and arrivals[pending[0]] <= t:
            waiting.append(pending.popleft())
        # admit in arrival order while the pool can hold the head request
        while waiting:
            k = waiting[0]
            r = requests[k]
            if backend.sim_bytes(r.params) > budget:
                rejected.append(r.rid)
                waiting.popleft()
                continue
            try:
                ticket = backend.admit(r.params, r.x0, r.m0, r.steps)
            except Exception:      # a failed request is dropped; the others go on
                rejected.append(r.rid)
                waiting.popleft()
                continue
            if ticket is None:
                break
            active[ticket] = (k, now())
            waiting.popleft()
        if active:
            backend.tick()
            ticks += 1
            for ticket in [tk for tk in active if backend.done(tk)]:
                k, t_adm = active.pop(ticket)
                r = requests[k]
                m, pairs = backend.result(ticket, int(r.params.n), int(getattr(r.params, "n_species", 1)))
                outcomes[r.rid] = Outcome(r.rid, arrivals[k], t_adm, now(), m, pairs)
        elif pending:
            gap = arrivals[pending[0]] - now()
            if gap > 0:
                if realtime:
                    sleep(min(gap, max_wait_s))
                else:
                    offset += gap
        elif waiting:
            # nothing active and the head does not fit an empty pool
            rejected.append(requests[waiting.popleft()].rid)
    return Report(outcomes, now(), ticks, rejected)
