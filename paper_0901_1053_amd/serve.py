"""Continuous-batching wake server.

Requests (a wake geometry, bunch and step count) arrive over time.  The server
keeps every admitted request's grid on the device and steps all of them with
one batch (tete_batch_*): a request is admitted, first come first served, as
soon as a batch slot is free and the HBM footprint of all admitted grids plus
its own stays within the budget; when its last wake sample is complete its
wake is copied to the host, its slot and memory are released, and the next
request is admitted.  Latency is measured from arrival to wake on the host.

The policy (admission, stepping, completion) is separate from the executor:
``GpuExecutor`` drives the HIP library, ``MockExecutor`` is a fake clock with a
cost model for testing the policy on the CPU.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

MAX_SLOTS = 256
HBM_BYTES = 288 * 10 ** 9


@dataclass
class Request:
    rid: int
    case: object                # inputs.WakeCase
    arrival: float              # seconds after the start of the run
    admitted: float = math.nan
    done: float = math.nan
    steps_left: int = 0
    slot: int = -1
    wake: np.ndarray | None = None
    footprint: int = 0

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def poisson_arrivals(rate: float, count: int, seed: int) -> np.ndarray:
    """Arrival times of a Poisson process of the given rate (seeded)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=float), q)) if len(xs) else math.nan


# ---------------------------------------------------------------------------
# Executors
# ---------------------------------------------------------------------------

class MockExecutor:
    """Fake clock: stepping k steps costs k * (cells of the active grids) / rate
    seconds plus a fixed overhead per call; set-up and read-back cost fixed
    times.  No GPU."""

    def __init__(self, rate_cells_per_s=5e10, step_overhead=2e-5, setup_s=1e-3, readout_s=2e-4):
        self.t = 0.0
        self.rate, self.step_overhead, self.setup_s, self.readout_s = rate_cells_per_s, step_overhead, setup_s, readout_s
        self.active = {}
        self.log = []

    def now(self) -> float:
        return self.t

    def wait_until(self, t: float):
        self.t = max(self.t, t)

    def footprint(self, case) -> int:
        return 12 * 4 * (case.nx + 1) * (case.ny + 1) * (case.nz + 1)

    def admit(self, slot, req):
        self.active[slot] = req
        self.t += self.setup_s
        self.log.append(("admit", slot, req.rid))

    def step(self, k):
        cells = sum(r.case.cells for r in self.active.values())
        self.t += k * cells / self.rate + self.step_overhead
        self.log.append(("step", k, len(self.active)))

    def finish(self, slot):
        req = self.active.pop(slot)
        self.t += self.readout_s
        self.log.append(("finish", slot, req.rid))
        return np.zeros(req.case.nw)

    def close(self):
        pass


class GpuExecutor:
    """Drives libtete: one Grid per request (workspace owned by torch), all of
    them members of one Batch; or, with batch=False, each request solved alone
    with tete_step (the one-at-a-time baseline)."""

    def __init__(self, precision="fp32", batch=True, graph_steps=8, tuner=None, device="cuda:0"):
        import torch

        from . import tete
        self.torch, self.tete = torch, tete
        self.precision = precision
        self.device = device
        self.tuner = tuner
        self.grids = {}
        self.batch = tete.Batch(precision, device=device) if batch else None
        if self.batch is not None:
            self.batch.set_launch(graph_steps=graph_steps)

    def now(self) -> float:
        return time.perf_counter()

    def wait_until(self, t: float):
        dt = t - time.perf_counter()
        if dt > 0:
            time.sleep(dt)

    def footprint(self, case) -> int:
        d = self.tete.make_desc(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.cdt, self.precision)
        return self.tete.workspace_bytes(d) + case.cells   # plus the staged cell mask

    def admit(self, slot, req):
        c = req.case
        G = self.tete.Grid(c.nx, c.ny, c.nz, c.dx, c.dy, c.dz, c.cdt, precision=self.precision, device=self.device)
        G.set_pec_cells(c.cell_mask())
        G.set_bunch(c.Q, c.sigma, c.i0, c.j0, c.M, c.jmin, c.nw)
        if self.tuner is not None:
            sh = self.tuner.lookup(c.nx, c.ny, c.nz, self.precision)
            if sh is not None:
                G.set_tuning(self.tuner.kernel, 0, sh.xchunk, 0, sh.order)   # the kernel it was timed on
        self.grids[slot] = G
        if self.batch is not None:
            self.batch.set(slot, G)

    def step(self, k):
        """Step every admitted request by k and wait until the block is done:
        at most one block is in flight, so a request that arrives meanwhile
        is admitted before the next block, not at the next completion."""
        if self.batch is not None:
            self.batch.step(k)
            stream = self.batch.stream
        else:
            for G in self.grids.values():
                G.step(k)
            stream = self.torch.cuda.current_stream(self.device)
        ev = self.torch.cuda.Event()
        ev.record(stream)
        ev.synchronize()

    def finish(self, slot):
        G = self.grids.pop(slot)
        w = G.wake()                      # synchronises
        if self.batch is not None:
            self.batch.set(slot, None)
        G.close()
        del G
        return w

    def close(self):
        for slot in list(self.grids):
            self.finish(slot)
        if self.batch is not None:
            self.batch.close()


# ---------------------------------------------------------------------------
# Policy
# ---------------------------------------------------------------------------

@dataclass
class ServeStats:
    completed: int
    makespan_s: float
    solves_per_s: float
    p50_s: float
    p99_s: float
    mean_s: float
    max_active: int
    peak_bytes: int
    latencies: list = field(default_factory=list)

    def as_dict(self):
        d = dict(self.__dict__)
        d.pop("latencies")
        return d


class Server:
    """First-come-first-served continuous batching.  A request is admitted when
    a slot is free, its HBM footprint fits the budget, and the grid cells in
    flight stay within max_cells (None: no limit; a request larger than the
    limit is admitted alone).  The cell limit keeps the device saturated
    without sharing it among more requests than needed, which would delay
    every one of them."""

    def __init__(self, executor, budget_bytes=HBM_BYTES - 16 * 10 ** 9, max_slots=MAX_SLOTS, block_steps=64,
                 max_cells=None):
        self.ex = executor
        self.budget = budget_bytes
        self.max_slots = max_slots
        self.block = block_steps
        self.max_cells = max_cells

    def run(self, requests) -> ServeStats:
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        for r in pending:
            r.footprint = self.ex.footprint(r.case)
            if r.footprint > self.budget:
                raise ValueError("request %d does not fit the HBM budget" % r.rid)
        active = {}
        free = list(range(self.max_slots))[::-1]
        used = 0
        cells = 0
        peak_bytes = 0
        max_active = 0
        t0 = self.ex.now()
        done = []
        while pending or active:
            now = self.ex.now() - t0
            # admit, first come first served, while a slot and the memory allow
            while (pending and pending[0].arrival <= now and free and used + pending[0].footprint <= self.budget
                   and (self.max_cells is None or not active or cells + pending[0].case.cells <= self.max_cells)):
                r = pending.popleft()
                r.slot = free.pop()
                used += r.footprint
                cells += r.case.cells
                peak_bytes = max(peak_bytes, used)
                self.ex.admit(r.slot, r)
                r.admitted = self.ex.now() - t0
                r.steps_left = r.case.steps
                active[r.slot] = r
                now = self.ex.now() - t0
            max_active = max(max_active, len(active))
            if not active:
                self.ex.wait_until(t0 + pending[0].arrival)
                continue
            # step until the next completion, or one block (new arrivals are
            # admitted between blocks)
            k = min(self.block, min(r.steps_left for r in active.values()))
            self.ex.step(k)
            for r in active.values():
                r.steps_left -= k
            for slot in [s for s, r in active.items() if r.steps_left == 0]:
                r = active.pop(slot)
                r.wake = self.ex.finish(slot)
                r.done = self.ex.now() - t0
                used -= r.footprint
                cells -= r.case.cells
                free.append(slot)
                done.append(r)
        makespan = max(r.done for r in done) if done else 0.0
        lat = [r.latency for r in done]
        return ServeStats(len(done), makespan, len(done) / makespan if makespan > 0 else math.nan,
                          percentile(lat, 50), percentile(lat, 99), float(np.mean(lat)) if lat else math.nan,
                          max_active, peak_bytes, lat)


def fifo_completions(arrivals, service):
    """Completion times of requests served one at a time, first come first
    served, by a server that is busy for service[i] seconds with request i."""
    done = []
    t = 0.0
    for a, s in zip(arrivals, service):
        t = max(t, a) + s
        done.append(t)
    return done


def one_at_a_time_stats(arrivals, service) -> ServeStats:
    """Statistics of one-at-a-time FIFO serving of a request stream, given
    each request's measured solve time alone (the server's behaviour does not
    depend on the arrival times otherwise, so one pass of solves serves every
    arrival rate)."""
    done = fifo_completions(arrivals, service)
    lat = [d - a for d, a in zip(done, arrivals)]
    makespan = max(done) if done else 0.0
    return ServeStats(len(done), makespan, len(done) / makespan if makespan > 0 else math.nan,
                      percentile(lat, 50), percentile(lat, 99), float(np.mean(lat)) if lat else math.nan,
                      1 if done else 0, 0, lat)


def solve_alone(executor, cases):
    """Each case solved alone through the executor (admit, all its steps,
    read-out, release), in order; returns (seconds per solve, wakes)."""
    times, wakes = [], []
    for i, c in enumerate(cases):
        r = Request(i, c, 0.0)
        t0 = executor.now()
        executor.admit(0, r)
        executor.step(c.steps)
        wakes.append(executor.finish(0))
        times.append(executor.now() - t0)
    return times, wakes


def make_requests(cases, rate, seed):
    arr = poisson_arrivals(rate, len(cases), seed)
    return [Request(i, c, float(t)) for i, (c, t) in enumerate(zip(cases, arr))]
