"""Serving scheduler (admission, retirement, latency accounting) against a
fake device: no GPU needed."""
import numpy as np
import pytest

from paper_2305_07030_amd import dr
from paper_2305_07030_amd import serve as SV


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeDevice:
    """Each solve needs a scripted number of passes; a tick advances every
    in-flight solve by the budget and costs `tick_cost` seconds."""

    def __init__(self, sizes, need, clock, tick_cost=1.0, cost=None):
        self.sizes = np.asarray(sizes)
        self.cost = cost
        self.need = need
        self.clock = clock
        self.tick_cost = tick_cost
        self.state = {}  # net -> [needed, done, result, F]
        self.launches = []

    def node_count(self, p):
        return int(self.sizes[p])

    def pass_cost(self, p):
        return 1.0 if self.cost is None else float(self.cost[p])

    def cost_min(self):
        return 1.0 if self.cost is None else float(min(self.cost))

    def advance(self, ids, starts, budgets, F):
        self.launches.append(list(map(int, ids)))
        self.budgets = dict(zip(map(int, ids), map(int, budgets)))
        for k, p in enumerate(ids):
            budget = int(budgets[k])
            p = int(p)
            if starts[k] == dr.DR_RESUME:
                st = self.state[p]
                assert st[2] == dr.DR_RUNNING
            else:
                st = self.state[p] = [self.need(p, F[k]), 0, dr.DR_RUNNING, np.array(F[k])]
            st[1] = min(st[0], st[1] + budget)
            if st[1] >= st[0]:
                st[2] = dr.DR_CONVERGED
        self.clock.t += self.tick_cost

    def query(self, ids):
        n = len(ids)
        res = np.array([self.state[int(p)][2] for p in ids], np.int32)
        it = np.array([self.state[int(p)][1] for p in ids], np.int64)
        sig = np.stack([self.state[int(p)][3] * 0.5 for p in ids])
        return dict(result=res, iters=it, sigma=sig, rho=np.zeros(n), ke=np.zeros(n),
                    sigma_fib=sig)


def make(sizes, need, budget_nodes, slots, tick=100):
    clock = FakeClock()
    dev = FakeDevice(sizes, need, clock)
    srv = SV.Server(dev, hbm_budget_bytes=SV.state_bytes_per_node() * budget_nodes,
                    max_slots=slots, tick_passes=tick, clock=clock)
    return clock, dev, srv


def test_admission_limits_and_one_request_per_network():
    sizes = [100, 200, 300, 400, 500, 600]
    clock, dev, srv = make(sizes, lambda p, F: 250 + 50 * p, budget_nodes=900, slots=3)
    stream = SV.RequestStream(np.tile(np.eye(3), (6, 1, 1)), rate=0.0, amp=0.002, seed=1)
    for _ in range(30):
        srv.submit(stream.make(0.0))
    seen_bytes, seen_slots = 0, 0
    while not srv.idle():
        srv.tick()
        seen_bytes = max(seen_bytes, srv.bytes_in_flight)
        seen_slots = max(seen_slots, len(srv.active))
        for launch in dev.launches:
            assert len(set(launch)) == len(launch)
        assert sum(sizes[p] for p in srv.active) * SV.state_bytes_per_node() == srv.bytes_in_flight
    assert len(srv.done) == 30
    assert seen_slots <= 3 and seen_bytes <= SV.state_bytes_per_node() * 900
    # every request of a network ran after the previous one of that network
    by_net = {}
    for r in srv.done:
        by_net.setdefault(r.net, []).append(r)
    for reqs in by_net.values():
        reqs.sort(key=lambda r: r.rid)
        for a, b in zip(reqs, reqs[1:]):
            assert b.t_admit >= a.t_done


def test_latency_accounting_and_passes():
    sizes = [10, 10]
    clock, dev, srv = make(sizes, lambda p, F: 350, budget_nodes=100, slots=4, tick=100)
    srv.submit(SV.Request(0, 0, np.eye(3), 0.0))
    srv.submit(SV.Request(1, 1, np.eye(3), 0.0))
    while not srv.idle():
        srv.tick()
    # 350 passes at 100 per tick = 4 ticks of 1 s each
    assert [r.t_done for r in srv.done] == [4.0, 4.0]
    assert [r.passes for r in srv.done] == [350, 350]
    assert all(r.result == dr.DR_CONVERGED for r in srv.done)


def test_budget_blocks_fifo_but_busy_network_does_not():
    sizes = [500, 500, 10]
    clock, dev, srv = make(sizes, lambda p, F: 100, budget_nodes=600, slots=8)
    srv.submit(SV.Request(0, 0, np.eye(3), 0.0))
    srv.submit(SV.Request(1, 0, np.eye(3), 0.0))   # same network: waits, does not block
    srv.submit(SV.Request(2, 2, np.eye(3), 0.0))   # fits in the budget beside request 0
    srv.submit(SV.Request(3, 1, np.eye(3), 0.0))   # would exceed the budget: waits
    srv.tick()
    assert sorted(r.rid for r in srv.done) == [0, 2]
    srv.tick()
    assert sorted(r.rid for r in srv.done) == [0, 1, 2]
    while not srv.idle():
        srv.tick()
    assert sorted(r.rid for r in srv.done) == [0, 1, 2, 3]


def test_oversized_request_rejected():
    clock, dev, srv = make([1000], lambda p, F: 10, budget_nodes=500, slots=2)
    with pytest.raises(ValueError):
        srv.submit(SV.Request(0, 0, np.eye(3), 0.0))


def test_request_stream_walks_F_symmetrically():
    s = SV.RequestStream(np.tile(np.eye(3), (4, 1, 1)), rate=10.0, amp=0.002, seed=7)
    rs = [s.make(0.0) for _ in range(50)]
    for r in rs:
        assert np.allclose(r.F, r.F.T)
    last = {}
    for r in rs:
        if r.net in last:
            assert np.abs(r.F - last[r.net]).max() <= 0.002 + 1e-15
        last[r.net] = r.F
    assert s.next_gap() > 0


def test_balanced_tick_budgets():
    """A tick lasts tick_passes passes of the pool's cheapest network; every
    in-flight solve makes as many passes as fit that time by its per-pass
    cost, whether or not the cheapest network is in flight."""
    clock = FakeClock()
    dev = FakeDevice([100, 200, 400, 50], lambda p, F: 10 ** 6, clock, cost=[1.0, 2.0, 4.0, 0.5])
    srv = SV.Server(dev, hbm_budget_bytes=SV.state_bytes_per_node() * 10 ** 6, max_slots=3,
                    tick_passes=800, clock=clock)
    for p in range(3):
        srv.submit(SV.Request(p, p, np.eye(3), 0.0))
    srv.tick()
    assert dev.budgets == {0: 400, 1: 200, 2: 100}
