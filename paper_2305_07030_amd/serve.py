"""Continuous-batching serving loop for many small dynamic-relaxation solves.

Simulated macroscale material points (the FE2 setting of section I) send
solve requests for the networks of a resident pool.  Each request names a
pool network and a new deformation gradient; it is warm-started from the
displacements the network's previous solve left on the device.

Scheduling is iteration-level continuous batching over the C ABI:
  * a request waits in a FIFO queue until it is admitted: a free slot, room in
    the HBM budget for its running state, and no other request of the same
    network in flight;
  * every tick is one dr_advance launch over all in-flight slots (new ones
    start warm, the others resume from their exact saved state) of a fixed
    length, tick_passes passes of the pool's cheapest network: every solve
    makes as many passes as fit that time (the library's per-pass cost
    estimates), so the launch's compute units finish together; requests that arrive while
    others run join the next launch and their work overlaps on the device;
  * after the tick dr_results reports which solves finished; those retire,
    free their slot and budget, and their latency (arrival to result on the
    host) is recorded.
A problem's arithmetic does not depend on what else is in the launch, so a
result is the same, bit for bit, alone and in the mix.

The device is any object with advance(ids, starts, budgets, F), query(ids),
node_count(p), pass_cost(p) and cost_min(); paper_2305_07030_amd.dr.DRBatch (wrapped by
PoolDevice) is the real one.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from . import dr


def state_bytes_per_node(precision: int = dr.DR_FP64) -> int:
    """Running state the device keeps per node of an in-flight solve (the
    library's own figure: two state records and one velocity record)."""
    return dr.state_bytes_per_node(precision)


@dataclass
class Request:
    rid: int
    net: int
    F: np.ndarray
    t_arrival: float
    t_admit: float = -1.0
    t_done: float = -1.0
    result: int = -1
    passes: int = 0
    sigma: Optional[np.ndarray] = None


@dataclass
class ServeStats:
    latencies: List[float] = field(default_factory=list)
    passes: List[int] = field(default_factory=list)
    results: List[int] = field(default_factory=list)
    completed: int = 0
    ticks: int = 0
    max_in_flight: int = 0
    max_bytes: int = 0
    wall: float = 0.0

    def summary(self) -> dict:
        lat = np.array(self.latencies) if self.latencies else np.zeros(1)
        return dict(completed=self.completed, ticks=self.ticks,
                    p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                    mean_s=float(lat.mean()), throughput_per_s=self.completed / max(self.wall, 1e-12),
                    max_in_flight=self.max_in_flight, max_state_bytes=self.max_bytes,
                    converged=int(sum(r == dr.DR_CONVERGED for r in self.results)))


class Server:
    def __init__(self, device, *, hbm_budget_bytes: int, max_slots: int, tick_passes: int,
                 clock: Callable[[], float] = time.perf_counter, bytes_per_node: Optional[int] = None):
        self.dev = device
        self.bytes_per_node = int(bytes_per_node or getattr(device, "bytes_per_node", 0)
                                  or state_bytes_per_node())
        self.budget = int(hbm_budget_bytes)
        self.max_slots = int(max_slots)
        self.tick_passes = int(tick_passes)
        self.clock = clock
        self.queue: collections.deque = collections.deque()
        self.active: Dict[int, Request] = {}  # net -> request in flight
        self.started: Dict[int, bool] = {}    # net -> launched at least once in this request
        self.bytes_in_flight = 0
        self.done: List[Request] = []

    def need_bytes(self, net: int) -> int:
        return self.bytes_per_node * int(self.dev.node_count(net))

    def submit(self, req: Request):
        if self.need_bytes(req.net) > self.budget:
            raise ValueError(f"network {req.net} alone exceeds the HBM budget")
        self.queue.append(req)

    def _admit(self, now: float):
        """FIFO admission; a request blocked by a busy network does not block
        the ones behind it, one blocked by slots or budget does."""
        kept = collections.deque()
        while self.queue:
            req = self.queue.popleft()
            if req.net in self.active:
                kept.append(req)
                continue
            nb = self.need_bytes(req.net)
            if len(self.active) >= self.max_slots or self.bytes_in_flight + nb > self.budget:
                kept.append(req)
                kept.extend(self.queue)
                self.queue.clear()
                break
            req.t_admit = now
            self.active[req.net] = req
            self.started[req.net] = False
            self.bytes_in_flight += nb
        self.queue = kept

    def tick(self) -> List[Request]:
        """One launch over all in-flight slots; returns the requests it finished."""
        self._admit(self.clock())
        if not self.active:
            return []
        nets = np.array(sorted(self.active), np.int32)
        starts = np.array([dr.DR_RESUME if self.started[n] else dr.DR_START_WARM for n in nets],
                          np.int32)
        F = np.stack([self.active[n].F for n in nets])
        cost = np.array([self.dev.pass_cost(int(n)) for n in nets])
        budgets = np.maximum(1, np.rint(self.tick_passes * self.dev.cost_min() / cost)).astype(np.int64)
        self.dev.advance(nets, starts, budgets, F=F)
        for n in nets:
            self.started[n] = True
        q = self.dev.query(nets)
        now = self.clock()
        finished = []
        for k, n in enumerate(nets):
            st = int(q["result"][k])
            if st == dr.DR_RUNNING:
                continue
            req = self.active.pop(int(n))
            self.started.pop(int(n))
            self.bytes_in_flight -= self.need_bytes(int(n))
            req.t_done = now
            req.result = st
            req.passes = int(q["iters"][k])
            req.sigma = np.array(q["sigma"][k])
            finished.append(req)
        self.done.extend(finished)
        return finished

    def idle(self) -> bool:
        return not self.active and not self.queue


class RequestStream:
    """Poisson arrivals naming uniform pool networks; each network's F walks:
    F <- F + a symmetric perturbation with entries U(-amp, amp)."""

    def __init__(self, F0: np.ndarray, rate: float, amp: float, seed: int):
        self.F = np.array(F0, dtype=np.float64).copy()
        self.rate = float(rate)
        self.amp = float(amp)
        self.rng = np.random.default_rng(np.random.SeedSequence(seed))
        self.rid = 0

    def next_gap(self) -> float:
        return float(self.rng.exponential(1.0 / self.rate)) if self.rate > 0 else 0.0

    def make(self, t: float) -> Request:
        p = int(self.rng.integers(0, len(self.F)))
        e = self.rng.uniform(-self.amp, self.amp, size=6)
        dF = np.array([[e[0], e[1], e[2]], [e[1], e[3], e[4]], [e[2], e[4], e[5]]])
        self.F[p] = self.F[p] + dF
        r = Request(self.rid, p, self.F[p].copy(), t)
        self.rid += 1
        return r


def run_open_loop(server: Server, stream: RequestStream, n_warmup: int, n_measure: int,
                  max_wall: float = 600.0) -> ServeStats:
    """Arrivals at stream.rate in wall-clock time; latencies of the n_measure
    requests after the first n_warmup are recorded."""
    stats = ServeStats()
    clock = server.clock
    t0 = clock()
    t_next = t0 + stream.next_gap()
    issued = 0
    total = n_warmup + n_measure
    while True:
        now = clock()
        while issued < total and t_next <= now:
            server.submit(stream.make(t_next))
            issued += 1
            t_next += stream.next_gap()
        if server.idle():
            if issued >= total:
                break
            time.sleep(max(0.0, min(t_next - clock(), 0.05)))
            continue
        fin = server.tick()
        stats.ticks += 1
        stats.max_in_flight = max(stats.max_in_flight, len(server.active))
        stats.max_bytes = max(stats.max_bytes, server.bytes_in_flight)
        for r in fin:
            if r.rid >= n_warmup:
                stats.latencies.append(r.t_done - r.t_arrival)
                stats.passes.append(r.passes)
                stats.results.append(r.result)
                stats.completed += 1
        if clock() - t0 > max_wall:
            break
    stats.wall = clock() - t0
    return stats


def run_closed_loop(server: Server, stream: RequestStream, n_requests: int,
                    max_wall: float = 600.0) -> ServeStats:
    """Keeps the queue full (every request arrives at once): the saturated
    solve rate of the device under this scheduler."""
    stats = ServeStats()
    clock = server.clock
    t0 = clock()
    for _ in range(n_requests):
        server.submit(stream.make(t0))
    while not server.idle():
        fin = server.tick()
        stats.ticks += 1
        stats.max_in_flight = max(stats.max_in_flight, len(server.active))
        stats.max_bytes = max(stats.max_bytes, server.bytes_in_flight)
        for r in fin:
            stats.latencies.append(r.t_done - r.t_arrival)
            stats.passes.append(r.passes)
            stats.results.append(r.result)
            stats.completed += 1
        if clock() - t0 > max_wall:
            break
    stats.wall = clock() - t0
    return stats


class PoolDevice:
    """The real device: a DRBatch over the pool plus its node counts."""

    def __init__(self, batch, **opts):
        self.batch = batch
        self.b = dr.DRBatch(batch, **opts)
        self.N = np.array([n.n_nodes for n in batch.nets])
        self.cost = self.b.pass_costs()
        self.bytes_per_node = state_bytes_per_node(opts.get("precision", dr.DR_FP64))

    def advance(self, ids, starts, budgets, F):
        self.b.advance(ids, starts, budgets, F=F)

    def pass_cost(self, p):
        return self.cost[p]

    def cost_min(self):
        return float(self.cost.min())

    def query(self, ids):
        return self.b.query(ids)

    def node_count(self, p):
        return self.N[p]
