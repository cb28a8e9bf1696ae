"""Continuous-batching serving on the GPU: a request's result is the same,
bit for bit, alone and in a mix of concurrent requests; warm starts match the
oracle's warm start."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2305_07030_amd import dr
from paper_2305_07030_amd import inputs as I
from paper_2305_07030_amd import serve as SV

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dr.load()
    O.build(force=False)


def pool():
    return I.small_batch(12, 80, 500, 0.0, seed=41)


def server(batch, slots=12):
    dev = SV.PoolDevice(batch, tol=1e-8, damping=1e-3, dt_safety=0.9)
    return SV.Server(dev, hbm_budget_bytes=SV.state_bytes_per_node() * 10 ** 7, max_slots=slots,
                     tick_passes=1500)


def test_alone_equals_in_the_mix():
    batch = pool()
    rng = np.random.default_rng(3)
    F_target = I.sym_perturbed_F(rng, 0.01)
    say("alone")
    s1 = server(batch)
    s1.submit(SV.Request(0, 3, F_target, 0.0))
    while not s1.idle():
        s1.tick()
    alone = s1.done[0]
    say("in a mix of 11 other requests arriving over several ticks")
    s2 = server(batch)
    others = [n for n in range(12) if n != 3]
    for k, n in enumerate(others[:5]):
        s2.submit(SV.Request(10 + k, n, I.sym_perturbed_F(rng, 0.01), 0.0))
    s2.tick()
    s2.tick()
    s2.submit(SV.Request(0, 3, F_target, 0.0))
    for k, n in enumerate(others[5:]):
        s2.submit(SV.Request(20 + k, n, I.sym_perturbed_F(rng, 0.01), 0.0))
    max_mix = 0
    while not s2.idle():
        s2.tick()
        max_mix = max(max_mix, len(s2.active))
    mixed = [r for r in s2.done if r.rid == 0][0]
    say("passes alone", alone.passes, "in mix", mixed.passes, "max in flight", max_mix)
    assert max_mix >= 6
    assert alone.result == mixed.result == dr.DR_CONVERGED
    assert alone.passes == mixed.passes
    assert np.array_equal(alone.sigma, mixed.sigma)


def test_warm_chain_matches_oracle():
    """Three successive requests to one network (each warm-started from the
    last result on the device) against the oracle's own warm chain."""
    batch = pool()
    net = batch.nets[5]
    Fs = [np.eye(3)]
    rng = np.random.default_rng(9)
    for _ in range(3):
        e = rng.uniform(-0.002, 0.002, 6)
        Fs.append(Fs[-1] + np.array([[e[0], e[1], e[2]], [e[1], e[3], e[4]], [e[2], e[4], e[5]]]))
    s = server(batch)
    u_prev, F_prev = None, None
    for k in range(1, 4):
        s.submit(SV.Request(k, 5, Fs[k], 0.0))
        while not s.idle():
            s.tick()
        g = s.done[-1]
        if u_prev is None:
            o = O.solve(net, Fs[k], tol=1e-8, beta=1e-3, dt_safety=0.9)
        else:
            o = O.solve(net, Fs[k], tol=1e-8, beta=1e-3, dt_safety=0.9, start=O.START_WARM,
                        F_prev=F_prev, u_prev=u_prev)
        u_prev, F_prev = o.u, Fs[k]
        err = np.linalg.norm(g.sigma - o.sigma) / np.linalg.norm(o.sigma)
        say(f"request {k}: passes gpu {g.passes} oracle {o.iters}, sigma rel {err:.2e}")
        assert g.result == dr.DR_CONVERGED
        assert err < 1e-7
