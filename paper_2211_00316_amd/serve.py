"""Serving: many reconstructions on one GPU with continuous batching.

A request is one scan to reconstruct: its ring, grid and ray fan, the measured data of its
frequencies (one frequency per step, low to high: the continuation of Section 6.3.2), and a
starting model. Requests arrive over time. The server admits a request as soon as the device
bytes it needs while running (rb_step_bytes of its geometry, plus its model) fit beside
those of the running requests within the HBM budget, first come first served; its model,
data, tables and operands stay on the GPU until its last step. Each round takes one
frequency step of every running request in one rb_frequency_step_batch call: the per-scan
stages of different scans overlap on the device, and their Born forward terms and
back-projections run as grouped launches. Requests therefore join and leave the batch at
step boundaries, and a request's result is the same whether it ran alone or in a mix.

The scheduling (Server) is host logic and is written against a small executor interface:
GpuExecutor drives the library; tests drive the same loop with a simulated executor.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np


@dataclasses.dataclass
class Request:
    """One reconstruction. omegas / d_omegas / windows: one entry per step. data: complex64
    [n_steps][n][n] in host memory (pinned for an asynchronous copy), copied to the device
    when the request is admitted and freed when it finishes; c_start: float64 [ny][nx]."""

    rid: int
    arrival: float
    grid: object
    ring: object
    tp: object
    omegas: list
    d_omegas: list
    windows: list
    data: object = None
    c_start: object = None
    tau: float = 0.12
    tag: str = ""
    # filled by the server
    c: object = None
    data_dev: object = None
    bytes: int = 0
    steps_done: int = 0
    status: int = 0
    t_admit: float = float("nan")
    t_done: float = float("nan")

    @property
    def n_steps(self) -> int:
        return len(self.omegas)

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


@dataclasses.dataclass
class Report:
    requests: list
    makespan: float
    steps: int
    batches: list            # number of scans in each batch, in order
    peak_bytes: int
    budget: int

    @property
    def steps_per_s(self) -> float:
        return self.steps / self.makespan if self.makespan > 0 else float("nan")

    def latency_pct(self, q) -> float:
        lat = [r.latency for r in self.requests if r.status == 0]
        return float(np.percentile(lat, q)) if lat else float("nan")

    def summary(self) -> dict:
        return {
            "requests": len(self.requests),
            "failed": sum(1 for r in self.requests if r.status != 0),
            "steps": self.steps,
            "makespan_s": round(self.makespan, 4),
            "steps_per_s": round(self.steps_per_s, 3),
            "p50_latency_s": round(self.latency_pct(50), 4),
            "p99_latency_s": round(self.latency_pct(99), 4),
            "mean_batch": round(float(np.mean(self.batches)), 3) if self.batches else 0.0,
            "max_batch": max(self.batches) if self.batches else 0,
            "peak_bytes": self.peak_bytes,
            "budget_bytes": self.budget,
        }


class Server:
    """Continuous batching over an executor with need_bytes(req), open(req), step(reqs) ->
    statuses, close(req). clock() and sleep(s) are injectable (simulated time in tests)."""

    def __init__(self, executor, budget_bytes: int, max_batch: int = 16,
                 clock=time.perf_counter, sleep=time.sleep, log=None):
        if max_batch < 1:
            raise ValueError("max_batch must be >= 1")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.clock = clock
        self.sleep = sleep
        self.log = log

    def run(self, requests) -> Report:
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        for r in pending:
            if r.n_steps < 1:
                raise ValueError(f"request {r.rid} has no step")
            r.bytes = int(self.ex.need_bytes(r))
            if r.bytes > self.budget:
                raise ValueError(f"request {r.rid} needs {r.bytes} bytes, above the budget "
                                 f"{self.budget}")
        active, batches, done = [], [], []
        used = peak = steps = 0
        t0 = self.clock()
        while pending or active:
            now = self.clock() - t0
            # admission: first come first served, while the head fits
            while (pending and pending[0].arrival <= now and len(active) < self.max_batch
                   and used + pending[0].bytes <= self.budget):
                r = pending.popleft()
                self.ex.open(r)
                r.t_admit = now
                used += r.bytes
                peak = max(peak, used)
                active.append(r)
            if not active:
                self.sleep(max(0.0, pending[0].arrival - (self.clock() - t0)))
                continue
            statuses = self.ex.step(active)
            now = self.clock() - t0
            batches.append(len(active))
            still = []
            for r, st in zip(active, statuses):
                if st == 0:
                    r.steps_done += 1
                    steps += 1
                else:
                    r.status = st
                if st != 0 or r.steps_done == r.n_steps:
                    r.t_done = now
                    self.ex.close(r)
                    used -= r.bytes
                    done.append(r)
                else:
                    still.append(r)
            active = still
            if self.log:
                self.log(f"t={now:.3f}s batch of {batches[-1]}, {len(done)} done, "
                         f"{len(pending)} waiting")
        return Report(sorted(done, key=lambda r: r.rid), self.clock() - t0, steps, batches, peak,
                      self.budget)


class GpuExecutor:
    """Runs the requests' steps with the library: one context per running request, on one of
    a few streams (default priority), with a tracer sample budget per request. A finished
    request's context is kept (its workspaces and mask lists stay allocated) and reused by
    the next request of the same geometry; kept contexts are destroyed when a new one would
    not fit beside them and the running requests within `budget` bytes."""

    def __init__(self, prec, device="cuda:0", n_streams: int = 4,
                 sample_budget: int = 12 << 30, budget: int | None = None, pool: bool = True):
        import torch

        from . import _lib

        self._lib = _lib
        self.torch = torch
        self.prec = prec
        self.device = device
        self.streams = [torch.cuda.Stream(device) for _ in range(n_streams)]
        self.sample_budget = int(sample_budget)
        self.budget = budget
        self.pool_on = pool
        self.ctx = {}
        self.active_bytes = 0
        self.pool = collections.OrderedDict()   # key -> list of (context, bytes), oldest first
        self._next = 0

    @staticmethod
    def _key(r):
        g, n, t = r.grid, r.ring, r.tp
        return (g.nx, g.ny, g.dx, g.x0, g.y0, g.mask_radius, n.n, n.radius, n.psi0, t.n_rays,
                t.max_steps, t.ds, t.c0)

    def pooled_bytes(self) -> int:
        return sum(b for lst in self.pool.values() for _, b in lst)

    def _evict(self, room: int):
        """Destroy kept contexts, oldest first, until `room` more bytes fit the budget."""
        while self.pool and self.budget is not None and \
                self.active_bytes + self.pooled_bytes() + room > self.budget:
            key = next(iter(self.pool))
            ctx, _ = self.pool[key].pop(0)
            if not self.pool[key]:
                del self.pool[key]
            ctx.close()

    def drain(self):
        """Destroy every kept context."""
        for lst in self.pool.values():
            for ctx, _ in lst:
                ctx.close()
        self.pool.clear()

    def _budget_for(self, r) -> int:
        # all emitters in one tracer launch when that fits, else chunks of the budget
        per_emitter = (r.tp.max_steps + 1) * r.tp.n_rays * 25
        return max(1 << 20, min(self.sample_budget, per_emitter * r.ring.n + (64 << 20)))

    def need_bytes(self, r) -> int:
        b = self._lib.step_bytes(r.grid, r.ring, r.tp, self.prec, self._budget_for(r))
        if b <= 0:
            raise ValueError(f"request {r.rid}: invalid geometry")
        model = 2 * r.grid.nx * r.grid.ny * 8   # model and its working copy
        data = r.n_steps * r.ring.n * r.ring.n * 8   # complex64 data of every step
        return b + model + data

    def open(self, r):
        torch = self.torch
        key = self._key(r)
        if self.pool.get(key):
            ctx, _ = self.pool[key].pop()
            if not self.pool[key]:
                del self.pool[key]
        else:
            self._evict(r.bytes)
            stream = self.streams[self._next % len(self.streams)]
            self._next += 1
            ctx = self._lib.Context(self.device, stream=stream)
            ctx.set_sample_budget(self._budget_for(r))
        self.active_bytes += r.bytes
        r.c = r.c_start.to(self.device, copy=True)
        r.data_dev = r.data.to(self.device, non_blocking=True)
        torch.cuda.current_stream().synchronize()   # the copies are done before the scan's stream reads them
        self.ctx[r.rid] = ctx

    def step(self, reqs):
        steps = []
        for r in reqs:
            k = r.steps_done
            steps.append(self._lib.ScanStep(
                self.ctx[r.rid], r.grid, r.ring, r.tp, r.c, r.windows[k], [r.omegas[k]],
                [r.d_omegas[k]], r.data_dev[k:k + 1], r.tau))
        return self._lib.frequency_step_batch(steps, self.prec)

    def close(self, r):
        ctx = self.ctx.pop(r.rid)
        self.active_bytes -= r.bytes
        r.data_dev = None   # the device copy of the data goes back to the allocator
        if self.pool_on:
            self.pool.setdefault(self._key(r), []).append((ctx, r.bytes))
        else:
            ctx.close()
