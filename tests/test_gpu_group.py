"""Workgroup groups and the tail hand-off, through the C ABI.

Once at most tail_at problems of a launch still run, they leave their
workgroups (exact state saved) and a cooperative launch finishes them with
several workgroups per problem.  Every node's arithmetic is the same as in
one workgroup, so at a fixed pass count the states are the same bits with the
hand-off and without it, whatever the number of workgroups per problem; the
group runs match the oracle node by node; a converged batch gives the same
results; budgets and energy terms carry over.
"""
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as O
from paper_2305_07030_amd import dr
from paper_2305_07030_amd import inputs as I

pytestmark = pytest.mark.gpu
S = 0.9


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


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


def mixed(seed, sizes, amp=0.02):
    rng = np.random.default_rng(seed)
    nets = [I.draw_network(rng, n) for n in sizes]
    return I.Batch(nets, np.stack([I.sym_perturbed_F(rng, amp) for _ in nets]))


def solve(batch, **kw):
    b = dr.DRBatch(batch, dt_safety=S, **kw)
    b.solve()
    r = b.results(want_u=True)
    b.close()
    return r


@pytest.mark.parametrize("precision", [dr.DR_FP64, dr.DR_FP32])
@pytest.mark.parametrize("group", [2, 4, 8, 16])
def test_fixed_passes_same_bits_any_group(precision, group):
    """Every problem hands off at pass 256 (tail_at = all of them) and makes
    the rest of its 1000 passes in a group of `group` workgroups: the same
    bits as without the hand-off.  Sizes span one row to several rows per
    wave of the group and both default classes (LDS and global)."""
    batch = mixed(41, [90, 700, 2600, 7100, 12000])
    K = 1000
    kw = dict(tol=1e-300, max_iter=K, damping=1e-3, precision=precision)
    ref = solve(batch, **kw)
    got = solve(batch, tail_at=len(batch), tail_group=group, **kw)
    say(f"precision {precision} group {group}: status {got['result'].tolist()}")
    assert (ref["result"] == dr.DR_MAX_ITER).all() and (got["result"] == dr.DR_MAX_ITER).all()
    assert np.array_equal(got["iters"], ref["iters"])
    assert np.array_equal(got["u"], ref["u"])
    assert np.array_equal(got["sigma"], ref["sigma"])


def oracle_fixed(net, F, K, beta):
    a = O.solve(net, F, tol=1e-30, max_iter=K, beta=beta, dt_safety=S)
    u0 = net.X @ (F - np.eye(3)).T
    u0 = u0 + np.random.default_rng(1).normal(size=u0.shape) * 1e-15 * (net.fixed == 0)[:, None]
    b = O.solve(net, F, tol=1e-30, max_iter=K, beta=beta, dt_safety=S, start=O.START_WARM,
                F_prev=F, u_prev=u0)
    return a, np.abs(a.u - b.u).max(), rel(b.sigma, a.sigma)


def test_group_runs_match_oracle_node_by_node():
    """A 33 000-node network and the two slowest networks of the 256-network
    workload (indices 103 and 24), run in groups of 8 after pass 256, against
    the oracle at a fixed pass count, node by node (the oracle's own
    sensitivity to a 1e-15 start perturbation sets the bar, as for the other
    placements)."""
    rng = np.random.default_rng(74)
    big = I.draw_network(rng, 33000)
    uni = I.config_uniform_batch(256, idx=[103, 24])
    batch = I.Batch([big] + uni.nets, np.concatenate([I.sym_perturbed_F(rng, 0.02)[None], uni.F]))
    K = 1500
    say("group runs vs oracle, N =", [n.n_nodes for n in batch.nets], f"{K} passes")
    g = solve(batch, tol=1e-30, max_iter=K, damping=1e-4, tail_at=len(batch), tail_group=8)
    with ThreadPoolExecutor(max_workers=3) as ex:
        ref = list(ex.map(lambda i: oracle_fixed(batch.nets[i], batch.F[i], K, 1e-4), range(3)))
    no = batch.packed()["node_offsets"]
    for i, (o, su, ss) in enumerate(ref):
        err = np.abs(g["u"][no[i]:no[i + 1]] - o.u).max()
        say(f"net {i} (N={batch.nets[i].n_nodes}): |du| {err:.2e} (sensitivity {su:.2e}), sigma rel "
            f"{rel(g['sigma'][i], o.sigma):.2e} (sensitivity {ss:.2e})")
        assert g["result"][i] == dr.DR_MAX_ITER and g["iters"][i] == K == o.iters
        assert err < 1e-12 + 100 * su
        assert rel(g["sigma"][i], o.sigma) < 1e-12 + 100 * ss


def test_converged_batch_with_hand_off():
    """A ragged batch solved to tol 1e-8 with the hand-off (the last 4
    problems finish in groups of 8): the same pass counts and stresses as
    without it, and the oracle's stresses within 1e-8."""
    batch = I.small_batch(24, 150, 1500, 0.02, seed=42)
    kw = dict(tol=1e-8, damping=1e-3)
    ref = solve(batch, **kw)
    got = solve(batch, tail_at=4, tail_group=8, **kw)
    say("passes", got["iters"].tolist())
    assert (got["result"] == dr.DR_CONVERGED).all()
    assert np.array_equal(got["iters"], ref["iters"])
    assert np.array_equal(got["sigma"], ref["sigma"])
    slow = np.argsort(got["iters"])[-4:]
    with ThreadPoolExecutor(max_workers=4) as ex:
        os_ = list(ex.map(lambda i: O.solve(batch.nets[i], batch.F[i], tol=1e-8, beta=1e-3, dt_safety=S),
                          slow))
    for i, o in zip(slow, os_):
        say(f"net {i}: passes {int(got['iters'][i])} (oracle {o.iters}), sigma rel {rel(got['sigma'][i], o.sigma):.2e}")
        assert rel(got["sigma"][i], o.sigma) < 1e-8


def test_budgeted_advance_with_hand_off():
    """dr_advance with a budget of 1000 passes: problems handed off at pass
    256 finish the budget in their group; the saved state then resumes
    (with and without the hand-off) to the same bits as one solve."""
    batch = mixed(43, [400, 1800, 5000, 9000])
    kw = dict(tol=1e-8, damping=1e-3, dt_safety=S)
    ref = dr.DRBatch(batch, **kw)
    ref.solve()
    R = ref.results()
    ref.close()
    ids = np.arange(len(batch), dtype=np.int32)
    b = dr.DRBatch(batch, tail_at=len(batch), tail_group=4, **kw)
    b.advance(ids, np.full(len(ids), dr.DR_START_AFFINE, np.int32), 1000, F=batch.F)
    q = b.query(ids)
    assert (q["result"] == dr.DR_RUNNING).all() and (q["iters"] == 1000).all()
    for k in range(100):
        run = ids[b.query(ids)["result"] == dr.DR_RUNNING]
        if len(run) == 0:
            break
        b.advance(run, np.full(len(run), dr.DR_RESUME, np.int32), 50000)
    q = b.query(ids)
    say("passes", q["iters"].tolist(), "reference", R["iters"].tolist())
    assert (q["result"] == dr.DR_CONVERGED).all()
    assert np.array_equal(q["iters"], R["iters"])
    assert np.array_equal(q["sigma"], R["sigma"])
    b.close()


def test_energy_terms_with_hand_off():
    batch = mixed(44, [300, 2500])
    kw = dict(tol=1e-300, max_iter=3000, damping=1e-3, energy_tol=0.5, dt_safety=S)
    a = dr.DRBatch(batch, **kw)
    a.solve()
    ra = a.results()
    ea = a.energy()
    b = dr.DRBatch(batch, tail_at=2, tail_group=4, **kw)
    b.solve()
    rb = b.results()
    eb = b.energy()
    assert np.array_equal(ra["sigma"], rb["sigma"]) and (rb["result"] == dr.DR_MAX_ITER).all()
    for k in ("work_int", "work_damp"):
        say(k, ea[k], eb[k])
        assert np.allclose(ea[k], eb[k], rtol=1e-12, atol=0)


def test_group_pass_time():
    """Time per pass of one 33 000-node network in global placement: one
    workgroup, then groups of 2 .. 16 (every pass after the first 256 in the
    group).  Printed for the record; the groups must not be slower than one
    workgroup."""
    rng = np.random.default_rng(75)
    batch = I.Batch([I.draw_network(rng, 33000)], I.sym_perturbed_F(rng, 0.02)[None])
    K = 4000
    times = {}
    for G in (1, 2, 4, 8, 16):
        kw = dict(tol=1e-300, max_iter=K, damping=1e-4, dt_safety=S, placement=dr.DR_PLACE_GLOBAL)
        if G > 1:
            kw.update(tail_at=1, tail_group=G)
        b = dr.DRBatch(batch, **kw)
        b.solve()
        b.results()
        t = time.perf_counter()
        b.solve()
        r = b.results()
        times[G] = (time.perf_counter() - t) / K * 1e6
        assert r["iters"][0] == K
        b.close()
    say("us per pass by workgroups per problem:", {k: round(v, 2) for k, v in times.items()})
    assert times[8] < times[1]
