"""Continuous-batching request loop over the batch engine.

Solve requests (grid, metric, layer, step count, and the initial spinor as
their payload) arrive over time.  The loop keeps one device arena (a torch uint8 tensor of `budget_bytes`)
and sub-allocates each admitted solve's buffer from it by its footprint
(``dirac_footprint_bytes``); a request is admitted as soon as it has arrived,
a batch slot is free and the arena has room, in arrival order.  Admitted solves
keep their state resident on the device until they finish.  Every quantum the
loop enqueues one batch run -- each running solve advances min(quantum, its
remaining steps) -- and, while that run is on the GPU, builds the tables of
newly arrived requests on a second stream, so new work joins at the next
quantum boundary.  Finished solves are copied out and their slot and memory are
released.  Latency = completion time - arrival time.

Solves in a batch run with a schedule that depends only on (n, precision), so
a request's result is bitwise the same whether it was served alone or in any
mix.
"""
from __future__ import annotations

import bisect
import time
from dataclasses import dataclass, field

import numpy as np

from . import dirac as D
from . import workloads as W


class Arena:
    """First-fit allocator over one device buffer (256-byte granules).

    With reserve=False the arena only does the bookkeeping of a budget (for
    budgets near the whole device, which cannot be reserved as one buffer); the
    caller then backs each granted block with its own allocation."""

    GRAN = 256

    def __init__(self, nbytes: int, device, reserve: bool = True):
        import torch
        self.nbytes = (nbytes // self.GRAN) * self.GRAN
        self.buffer = torch.empty(self.nbytes, dtype=torch.uint8, device=device) if reserve else None
        self.base = self.buffer.data_ptr() if reserve else None
        self.free = [(0, self.nbytes)]          # sorted (offset, size)
        self.used = 0

    def alloc(self, size: int):
        size = -(-size // self.GRAN) * self.GRAN
        for i, (off, sz) in enumerate(self.free):
            if sz >= size:
                if sz == size:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + size, sz - size)
                self.used += size
                return off, size
        return None

    def release(self, off: int, size: int):
        self.used -= size
        i = bisect.bisect_left(self.free, (off, 0))
        self.free.insert(i, (off, size))
        # merge with neighbours
        merged = []
        for o, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free = merged


@dataclass
class Request:
    rid: int
    arrival: float
    spec: W.SolveSpec
    steps: int
    psi0: np.ndarray | None = None       # initial spinor payload; built from the spec at admission if None
    admitted: float = -1.0
    finished: float = -1.0
    result: np.ndarray | None = None
    obs: dict | None = None


@dataclass
class _Running:
    req: Request
    solver: "D.Solver"
    slot: int
    off: int
    size: int
    remaining: int


class _ArenaSolver(D.Solver):
    """A Solver whose device buffer is a slice of the arena (ptr), or a buffer of
    its own when the arena only accounts (ptr None)."""

    def __init__(self, spec, precision, ptr, nbytes, stream):
        import torch
        self.n1, self.n2, self.precision = spec.n1, spec.n2, precision
        self.grid, self.metric, self.pml, keep = D.spec_structs(spec)
        self.nbytes = nbytes
        self.stream = stream
        self.buffer = None
        if ptr is None:
            self.buffer = torch.empty(nbytes, dtype=torch.uint8, device=stream.device)
            ptr = self.buffer.data_ptr()
        self.h = None
        self.h = D.create_metric(self.grid, self.metric, self.pml, precision, ptr, nbytes, stream.cuda_stream)
        del keep


@dataclass
class ServeStats:
    requests: int
    wall_s: float
    point_steps: float
    throughput: float
    p50_s: float
    p99_s: float
    mean_s: float
    max_running: int
    quanta: int
    budget_bytes: int
    peak_arena_bytes: int
    latencies: list = field(default_factory=list)


class Server:
    def __init__(self, precision=D.FP32, budget_bytes=288 << 30, capacity=512, quantum=64, keep_results=False,
                 device=None, policy="share", fill_points=1 << 22):
        import torch
        self.precision = precision
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        # budgets beyond 64 GiB are accounted, not reserved: each admitted solve then
        # gets its own buffer from torch's caching allocator
        self.reserve = budget_bytes <= (64 << 30)
        self.arena = Arena(budget_bytes, self.device, reserve=self.reserve)
        self.batch_stream = torch.cuda.Stream(self.device)
        self.setup_stream = torch.cuda.Stream(self.device)
        self.batch = D.Batch(precision=precision, capacity=capacity, device=self.device, stream=self.batch_stream)
        self.capacity = capacity
        self.quantum = quantum
        self.keep_results = keep_results
        if policy not in ("share", "srpt"):
            raise ValueError("policy must be 'share' or 'srpt'")
        self.policy = policy
        self.fill_points = fill_points

    def _plan(self, running):
        """Steps per running solve for the next quantum.  share: every solve advances.
        srpt: solves in order of least remaining work (grid points x steps left) until
        their grid points reach fill_points (enough to keep the device busy); the
        others wait for a later quantum."""
        if self.policy == "share":
            return {sl: min(self.quantum, ru.remaining) for sl, ru in running.items()}
        order = sorted(running.items(),
                       key=lambda kv: (kv[1].remaining * kv[1].req.spec.n1 * kv[1].req.spec.n2, kv[1].req.rid))
        steps, points = {}, 0
        for sl, ru in order:
            if steps and points >= self.fill_points:
                break
            steps[sl] = min(self.quantum, ru.remaining)
            points += ru.req.spec.n1 * ru.req.spec.n2
        return steps

    def _ptr(self, off):
        return None if self.arena.base is None else self.arena.base + off

    def _footprint(self, spec):
        g, m, p, _ = D.spec_structs(spec)
        return D.footprint_bytes(g, m, p, self.precision)

    def run(self, requests: list[Request], time_scale: float = 1.0) -> ServeStats:
        """Serve requests whose `arrival` times are seconds from the start (scaled by
        time_scale).  Returns latency and throughput statistics."""
        pending = sorted(requests, key=lambda r: r.arrival)
        for r in pending:
            if self._footprint(r.spec) > self.arena.nbytes:
                raise ValueError(f"request {r.rid} needs more than the whole budget")
        running: dict[int, _Running] = {}
        done: list[Request] = []
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        peak = 0
        max_running = 0
        quanta = 0
        qi = 0
        def admit():
            # admit everything that has arrived and fits (arrival order, no overtaking)
            nonlocal qi
            while qi < len(pending) and pending[qi].arrival * time_scale <= now() and len(running) < self.capacity:
                r = pending[qi]
                got = self.arena.alloc(self._footprint(r.spec))
                if got is None:
                    break
                off, size = got
                s = _ArenaSolver(r.spec, self.precision, self._ptr(off), size, self.setup_stream)
                s.set_initial_spinor(r.psi0 if r.psi0 is not None else W.initial_spinor(r.spec))
                slot = self.batch.add(s)
                r.admitted = now()
                running[slot] = _Running(r, s, slot, off, size, r.steps)
                qi += 1

        while qi < len(pending) or running:
            admit()
            peak = max(peak, self.arena.used)
            max_running = max(max_running, len(running))
            if not running:
                # idle: wait for the next arrival
                if qi < len(pending):
                    wait = pending[qi].arrival * time_scale - now()
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
                continue
            steps = self._plan(running)
            self.batch.run(steps)
            quanta += 1
            # while the quantum runs, admit newly arrived requests (their setup runs on
            # the setup stream and overlaps the batch stream)
            admit()
            self.batch.sync()
            t_done = now()
            for sl, st in steps.items():
                ru = running[sl]
                ru.remaining -= st
                if ru.remaining == 0:
                    r = ru.req
                    r.finished = t_done
                    if self.keep_results:
                        r.result = ru.solver.get_spinor()
                        r.obs = ru.solver.observables()
                    self.batch.remove(sl)
                    ru.solver.close()
                    self.arena.release(ru.off, ru.size)
                    del running[sl]
                    done.append(r)
            peak = max(peak, self.arena.used)
        wall = now()
        lat = sorted(r.finished - r.arrival * time_scale for r in done)
        work = float(sum(r.spec.n1 * r.spec.n2 * r.steps for r in done))
        pick = lambda q: lat[min(len(lat) - 1, int(round(q * (len(lat) - 1))))]
        return ServeStats(len(done), wall, work, work / wall, pick(0.5), pick(0.99), float(np.mean(lat)),
                          max_running, quanta, self.arena.nbytes, peak, lat)

    def close(self):
        self.batch.close()


def make_requests(count: int, rate_per_s: float, seed: int = 5000, sizes=(64, 128, 256, 512, 1024),
                  steps_range=(200, 5000), payload: bool = True) -> list[Request]:
    """Poisson arrivals of packet solves.  payload: each request carries its initial
    spinor, as a client would send it (else the server builds it at admission)."""
    out = []
    for i, (t, spec) in enumerate(W.serving_arrivals(count, rate_per_s, seed, sizes, steps_range)):
        out.append(Request(i, t, spec, spec.steps, W.initial_spinor(spec) if payload else None))
    return out
