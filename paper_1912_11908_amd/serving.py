"""Continuous-batching server for many independent solves on one GPU.

Requests (arrival time, case) arrive over wall-clock time.  The loop admits
arrived requests in FIFO order while the device-memory budget and the
active-solve cap allow, advances every active solve by one tick of steps
through the batched entry point (each stage of all stationary solves of one
kind is a single launch), retires solves that have finished, and records
each solve's latency from arrival to the completion of its last step.  One
tick is kept in flight: the host prepares and enqueues tick k+1 while the
GPU runs tick k, and stamps completions when a tick's event has fired.

The policy is independent of the device: ``GpuBackend`` drives the library;
tests drive the same loop with a simulated backend.
"""
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Job:
    rid: int
    arrival: float
    case: object
    steps_left: int
    evals: int                     # cell-updates of the whole solve
    need: int                      # device bytes while active
    start: float = -1.0
    done: float = -1.0
    solver: object = None
    status: int = 0


@dataclass
class Stats:
    latencies: list = field(default_factory=list)
    cell_updates: float = 0.0
    wall: float = 0.0
    max_active: int = 0
    ticks: int = 0
    failed: int = 0

    def summary(self):
        lat = np.asarray(self.latencies, dtype=float)
        return {
            "requests": int(lat.size),
            "p50_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_s": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_s": float(lat.mean()) if lat.size else None,
            "cell_updates": float(self.cell_updates),
            "wall_s": float(self.wall),
            "cell_updates_per_s": float(self.cell_updates / self.wall) if self.wall > 0 else None,
            "max_active": int(self.max_active),
            "ticks": int(self.ticks),
            "failed": int(self.failed),
        }


def case_cell_updates(case):
    """Cell-updates of a whole solve: cells x residual evaluations."""
    return case.ncells * case.evals_per_step * case.steps


class Server:
    """FIFO admission under `mem_budget` bytes and `max_active` solves.
    Every tick advances each active solve by about `tick_evals` residual
    evaluations (its steps per tick: tick_evals over its evaluations per
    step, at least one, at most the steps it has left); solves advancing by
    the same number of steps share one batched call."""

    def __init__(self, backend, mem_budget, max_active=128, tick_evals=30):
        self.backend = backend
        self.mem_budget = int(mem_budget)
        self.max_active = int(max_active)
        self.tick_evals = int(tick_evals)

    def steps_per_tick(self, job):
        k = max(1, self.tick_evals // int(job.case.evals_per_step))
        return min(k, job.steps_left)

    def run(self, requests):
        be = self.backend
        pending = deque()
        for rid, (t, case) in enumerate(requests):
            pending.append(Job(rid, float(t), case, int(case.steps), case_cell_updates(case),
                               be.bytes_needed(case)))
        for j in pending:
            if j.need > self.mem_budget:
                raise ValueError(f"request {j.rid} needs {j.need} bytes, over the budget")
        active, inflight, stats = [], deque(), Stats()
        used = 0
        t0 = be.now()
        while pending or active or inflight:
            now = be.now() - t0
            # admission: FIFO while memory and the cap allow
            while (pending and pending[0].arrival <= now and len(active) < self.max_active
                   and used + pending[0].need <= self.mem_budget):
                j = pending.popleft()
                j.solver = be.create(j.case)
                j.start = now
                used += j.need
                active.append(j)
            stats.max_active = max(stats.max_active, len(active))
            if active:
                by_k = {}
                for j in active:
                    by_k.setdefault(self.steps_per_tick(j), []).append(j)
                for k, jobs in sorted(by_k.items()):
                    be.advance([j.solver for j in jobs], k)
                    for j in jobs:
                        j.steps_left -= k
                finished = [j for j in active if j.steps_left == 0]
                active = [j for j in active if j.steps_left > 0]
                for j in finished:
                    be.finish(j.solver)
                inflight.append((be.mark(), finished))
                stats.ticks += 1
            elif not inflight:
                # idle: wait for the next arrival
                be.sleep_until(t0 + pending[0].arrival)
                continue
            # keep one tick in flight: wait for the older one
            while len(inflight) > (1 if active else 0):
                ev, finished = inflight.popleft()
                be.wait(ev)
                tdone = be.now() - t0
                for j in finished:
                    j.done = tdone
                    j.status = be.status(j.solver)
                    stats.failed += j.status != 0
                    stats.latencies.append(j.done - j.arrival)
                    stats.cell_updates += j.evals
                    used -= j.need
                    be.release(j.solver)
                    j.solver = None
        stats.wall = be.now() - t0
        return stats


class GpuBackend:
    """Solves on one GPU through the C ABI (Solver + batch_advance), on
    non-blocking streams of their own, so that creating a solve (which
    uploads its geometry synchronously) never waits for the batch in flight.
    RK3 and dual-time solves run on two streams, so the launch chains of the
    two kinds overlap; a solve always stays on its kind's stream, and its
    memory is released only after both streams' tick events have fired."""

    def __init__(self, precision="mixed", device="cuda:0", init=None):
        import torch
        from . import Solver, batch_advance, workspace_bytes, BATCH_MAX
        self.torch = torch
        self.Solver = Solver
        self.batch_advance = batch_advance
        self.workspace_bytes = workspace_bytes
        self.batch_max = BATCH_MAX
        self.precision = precision
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(self.device)
        self.streams = {"rk3": self.stream, "dual": torch.cuda.Stream(self.device)}
        self.init = init

    def bytes_needed(self, case):
        nv = case.ndim + 2
        hz = 3 if case.ndim == 3 else 0
        state = nv * (case.nk + 2 * hz) * (case.nj + 6) * (case.ni + 6) * 8
        return int(self.workspace_bytes(case, self.precision)) + state

    def create(self, case):
        torch = self.torch
        st = self.streams[case.scheme]
        with torch.cuda.stream(st):
            s = self.Solver(case, self.precision, str(self.device), stream=st)
            if self.init is not None:
                prim = torch.from_numpy(self.init(case)).pin_memory()
                s.init_prim(prim.to(self.device, non_blocking=True))
        s._serving_stream = st
        return s

    def advance(self, solvers, k):
        by_stream = {}
        for s in solvers:
            by_stream.setdefault(id(s._serving_stream), (s._serving_stream, []))[1].append(s)
        for st, group in by_stream.values():
            for m in range(0, len(group), self.batch_max):
                self.batch_advance(group[m:m + self.batch_max], k, stream=st)

    def mark(self):
        evs = []
        for st in self.streams.values():
            ev = self.torch.cuda.Event()
            ev.record(st)
            evs.append(ev)
        return evs

    def wait(self, evs):
        for ev in evs:
            ev.synchronize()

    def finish(self, solver):
        """Enqueue the copy of the solve's status word to pinned host memory
        (read by status() once the tick's event has fired)."""
        torch = self.torch
        off = solver.info().counts - solver.workspace.data_ptr()
        solver._status_host = torch.empty(8, dtype=torch.int32, pin_memory=True)
        with torch.cuda.stream(solver._serving_stream):
            src = solver.workspace[off:off + 32].view(torch.int32)
            solver._status_host.copy_(src, non_blocking=True)

    def status(self, solver):
        """0, or the library's IBM_ECAPACITY / IBM_ENONFINITE code."""
        word = int(solver._status_host[5])
        if word & 2:
            return -6
        if word & 1:
            return -4
        return 0

    def release(self, solver):
        del solver

    def now(self):
        return time.perf_counter()

    def sleep_until(self, t):
        dt = t - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
