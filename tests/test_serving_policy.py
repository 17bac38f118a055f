"""Continuous-batching policy of the server, driven by a simulated backend
(no GPU): every request completes with exactly its steps, admission is FIFO
under the memory budget and the active-solve cap, one tick stays in flight,
and the latency percentiles are those of the recorded latencies."""
from dataclasses import dataclass

import numpy as np
import pytest

from paper_1912_11908_amd.serving import Server, case_cell_updates


@dataclass
class FakeCase:
    ncells: int
    steps: int
    evals_per_step: int = 3
    ndim: int = 2


class SimBackend:
    """Time advances with the work enqueued: rate cell-updates per second,
    plus a fixed cost per batched call."""

    def __init__(self, rate=1e9, per_call=1e-4):
        self.t = 0.0
        self.gpu_free = 0.0
        self.rate = rate
        self.per_call = per_call
        self.steps_done = {}
        self.used = 0
        self.max_used = 0
        self.active = set()
        self.max_active = 0
        self.admitted = []
        self.inflight_max = 0
        self.pending_marks = []
        self.max_batch = 0

    def bytes_needed(self, case):
        return case.ncells * 100

    def create(self, case):
        sid = len(self.admitted)
        self.admitted.append(case)
        self.steps_done[sid] = 0
        self.used += self.bytes_needed(case)
        self.max_used = max(self.max_used, self.used)
        self.active.add(sid)
        self.max_active = max(self.max_active, len(self.active))
        return sid

    def advance(self, solvers, k):
        self.max_batch = max(self.max_batch, len(solvers))
        work = sum(self.admitted[s].ncells * self.admitted[s].evals_per_step * k for s in solvers)
        start = max(self.t, self.gpu_free)
        self.gpu_free = start + self.per_call + work / self.rate
        for s in solvers:
            self.steps_done[s] += k

    def finish(self, solver):
        pass

    def mark(self):
        self.pending_marks.append(self.gpu_free)
        self.inflight_max = max(self.inflight_max, len(self.pending_marks))
        return self.gpu_free

    def wait(self, ev):
        self.t = max(self.t, ev)
        self.pending_marks.remove(ev)

    def status(self, solver):
        return 0

    def release(self, solver):
        self.used -= self.bytes_needed(self.admitted[solver])
        self.active.discard(solver)

    def now(self):
        self.t += 1e-6
        return self.t

    def sleep_until(self, t):
        self.t = max(self.t, t)


def _requests(n=60, rate=50.0, seed=3):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    sides = rng.choice([64, 128, 256], n)
    steps = rng.integers(5, 40, n)
    return [(float(t[m]), FakeCase(int(sides[m]) ** 2, int(steps[m]))) for m in range(n)]


def test_every_request_completes_with_its_steps():
    reqs = _requests()
    be = SimBackend()
    st = Server(be, mem_budget=10 ** 9, max_active=16, tick_evals=21).run(reqs)
    assert len(st.latencies) == len(reqs)
    assert [be.steps_done[m] for m in range(len(reqs))] == [c.steps for _, c in reqs]
    assert st.cell_updates == sum(case_cell_updates(c) for _, c in reqs)
    assert all(lat > 0 for lat in st.latencies)
    assert be.inflight_max <= 2


def test_memory_budget_and_cap_hold():
    reqs = _requests(80, rate=400.0)
    be = SimBackend(rate=2e8)
    budget = 256 * 256 * 100 * 3
    st = Server(be, mem_budget=budget, max_active=5, tick_evals=12).run(reqs)
    assert be.max_used <= budget          # finished solves hold memory until their tick ends
    assert be.max_batch <= 5
    assert len(st.latencies) == len(reqs)
    # FIFO: solves are created in arrival order
    assert [c.ncells for c in be.admitted] == [c.ncells for _, c in reqs]


def test_oversized_request_rejected():
    reqs = [(0.0, FakeCase(512 * 512, 3))]
    with pytest.raises(ValueError):
        Server(SimBackend(), mem_budget=1000).run(reqs)


def test_percentiles_match_latencies():
    reqs = _requests(40)
    st = Server(SimBackend(), mem_budget=10 ** 9).run(reqs)
    s = st.summary()
    lat = np.array(st.latencies)
    assert s["p50_s"] == pytest.approx(np.percentile(lat, 50))
    assert s["p99_s"] == pytest.approx(np.percentile(lat, 99))
    assert s["requests"] == 40


def test_ticks_equalise_evaluations():
    """A solve with 20 evaluations per step advances one step per tick while
    3-evaluation solves advance tick_evals / 3 steps."""
    reqs = [(0.0, FakeCase(64 * 64, 40)), (0.0, FakeCase(64 * 64, 4, evals_per_step=20))]
    be = SimBackend()
    calls = []
    orig = be.advance

    def rec(solvers, k):
        calls.append((tuple(solvers), k))
        orig(solvers, k)
    be.advance = rec
    st = Server(be, mem_budget=10 ** 9, tick_evals=30).run(reqs)
    assert len(st.latencies) == 2
    assert ((0,), 10) in calls and ((1,), 1) in calls
    assert be.steps_done == {0: 40, 1: 4}


def test_latency_at_least_the_solve_alone():
    """Under light load a request's latency is its own solve time plus at
    most one tick of admission delay."""
    reqs = [(m * 10.0, FakeCase(128 * 128, 20)) for m in range(5)]
    be = SimBackend(rate=1e9, per_call=0.0)
    st = Server(be, mem_budget=10 ** 9, tick_evals=15).run(reqs)
    alone = 128 * 128 * 3 * 20 / 1e9
    for lat in st.latencies:
        assert alone * 0.999 <= lat <= alone * 1.5 + 1e-3
