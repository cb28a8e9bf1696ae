"""The per-pass time step (dt_rule 1: Fig. 1's "compute next time step" from
the current stiffness, never growing back), through the C ABI.

- Where every step stays the constant one it gives the constant-step bits.
- Where the rule acts (fibers stretched beyond the constant step's headroom)
  the GPU runs the oracle's iteration: node by node at a fixed pass count
  (bar: 100x the oracle's own sensitivity to a 1e-15 start perturbation, as
  for the other kernels), the chain's bisection equilibrium at convergence.
- A solve split over budgeted launches equals one launch, bit for bit.
- The networks of the 1024-network workload whose constant-step solves
  diverge converge with it: to a state the oracle's own residual certifies
  as an equilibrium, with the oracle's stress (stored oracle results).
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle as O
from paper_2305_07030_amd import dr
from paper_2305_07030_amd import inputs as I

pytestmark = pytest.mark.gpu
S = 0.9
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


def solve(batch, start=dr.DR_START_AFFINE, **kw):
    b = dr.DRBatch(batch, dt_safety=S, **kw)
    b.solve(start=start)
    r = b.results(want_u=True)
    b.close()
    return r


def test_same_bits_where_the_step_stays_constant():
    """A ragged batch (one to several slices, several rows per wave at 256
    threads) from the affine start: every fiber stays within the headroom,
    the step stays dt0, and the per-pass kernel gives the constant-step
    kernels' bits (which are the same for every launch shape)."""
    rng = np.random.default_rng(91)
    nets = [I.draw_network(rng, n) for n in (70, 700, 2600, 7100)]
    batch = I.Batch(nets, np.stack([I.sym_perturbed_F(rng, 0.02) for _ in nets]))
    for kw in (dict(tol=1e-8, damping=1e-3), dict(tol=1e-300, max_iter=1500, damping=1e-4)):
        ref = solve(batch, **kw)
        for block in (256, 1024):
            got = solve(batch, dt_rule=1, block=block, **kw)
            say(f"{kw} block {block}: passes {got['iters'].tolist()}")
            assert np.array_equal(got["iters"], ref["iters"])
            assert np.array_equal(got["result"], ref["result"])
            assert np.array_equal(got["u"], ref["u"])
            assert np.array_equal(got["sigma"], ref["sigma"])


def stretched_batch():
    """Small kNN networks relaxed from u = 0 under a 30 % stretch: most
    fibers start far beyond the constant step's headroom (the constant-step
    solve diverges on most of them)."""
    b = I.small_batch(3, 150, 400, 0.02, seed=81)
    return I.Batch(b.nets, np.stack([np.diag([1.3, 1.0, 1.0])] * 3))


def test_fixed_passes_match_oracle_where_the_rule_acts():
    batch = stretched_batch()
    K = 300
    g = solve(batch, start=dr.DR_START_ZERO, dt_rule=1, tol=1e-300, max_iter=K, damping=1e-3)
    no = batch.packed()["node_offsets"]
    for i, (net, F) in enumerate(zip(batch.nets, batch.F)):
        o = O.solve(net, F, tol=1e-30, max_iter=K, beta=1e-3, dt_safety=S, start=O.START_ZERO, dt_rule=1)
        u0 = np.where(net.fixed[:, None] == 1, net.X @ (F - np.eye(3)).T, 0.0)
        u0 = u0 + np.random.default_rng(1).normal(size=u0.shape) * 1e-15 * (net.fixed == 0)[:, None]
        p = O.solve(net, F, tol=1e-30, max_iter=K, beta=1e-3, dt_safety=S, start=O.START_WARM,
                    F_prev=F, u_prev=u0, dt_rule=1)
        sens = np.abs(p.u - o.u).max()
        err = np.abs(g["u"][no[i]:no[i + 1]] - o.u).max()
        say(f"net {i} (N={net.n_nodes}): smallest step {o.dt_min / o.dt:.3f} dt0, |du| {err:.2e} "
            f"(sensitivity {sens:.2e}), sigma rel {rel(g['sigma'][i], o.sigma):.2e}")
        assert o.dt_min < 0.9 * o.dt  # the rule acted
        assert g["result"][i] == dr.DR_MAX_ITER and g["iters"][i] == K
        assert err < 1e-12 + 100 * sens
        assert rel(g["sigma"][i], o.sigma) < 1e-12 + 100 * rel(p.sigma, o.sigma)


def test_stretched_chain_converges_to_bisection():
    """The collinear chain stretched four-fold from u = 0: the constant step
    diverges, the per-pass step converges to the equilibrium found by
    bisection."""
    X = np.array([[0.2, 0.5, 0.5], [0.45, 0.5, 0.5], [0.8, 0.5, 0.5]])
    net = I.Network(X, np.array([[0, 1], [1, 2]], np.int32), np.array([1.0, 1.7]),
                    np.array([1, 0, 1], np.uint8))
    F = np.diag([4.0, 1.0, 1.0])
    batch = I.Batch([net], F[None])
    a = solve(batch, start=dr.DR_START_ZERO, tol=1e-12, damping=0.05)
    b = solve(batch, start=dr.DR_START_ZERO, dt_rule=1, tol=1e-12, damping=0.05)
    assert a["result"][0] == dr.DR_NONFINITE
    assert b["result"][0] == dr.DR_CONVERGED
    # equilibrium: EA1 (l1^2/L1^2 - 1) = EA2 (l2^2/L2^2 - 1), l1 + l2 = 4 * 0.6
    L1, L2, ell = 0.25, 0.35, 4.0 * 0.6
    lo, hi = 1e-9, ell - 1e-9
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        h = 1.0 * ((mid / L1) ** 2 - 1) - 1.7 * (((ell - mid) / L2) ** 2 - 1)
        lo, hi = (lo, mid) if h > 0 else (mid, hi)
    xB = 4.0 * 0.2 + 0.5 * (lo + hi)
    assert abs(X[1, 0] + b["u"][1, 0] - xB) < 1e-11
    o = O.solve(net, F, tol=1e-12, beta=0.05, dt_safety=S, start=O.START_ZERO, dt_rule=1)
    say(f"chain: passes GPU {int(b['iters'][0])}, oracle {o.iters}")
    assert abs(int(b["iters"][0]) - o.iters) <= 1


def test_budgeted_launches_equal_one_launch():
    batch = stretched_batch()
    kw = dict(tol=1e-8, damping=1e-3, dt_safety=S, dt_rule=1)
    ref = dr.DRBatch(batch, **kw)
    ref.solve(start=dr.DR_START_ZERO)
    R = ref.results()
    ref.close()
    ids = np.arange(len(batch), dtype=np.int32)
    b = dr.DRBatch(batch, **kw)
    b.advance(ids, np.full(len(ids), dr.DR_START_ZERO, np.int32), 700, F=batch.F)
    for _ in range(1000):
        run = ids[b.query(ids)["result"] == dr.DR_RUNNING]
        if len(run) == 0:
            break
        b.advance(run, np.full(len(run), dr.DR_RESUME, np.int32), 3000)
    q = b.query(ids)
    b.close()
    say("passes", q["iters"].tolist(), "one launch", R["iters"].tolist())
    assert (R["result"] == dr.DR_CONVERGED).all()
    assert np.array_equal(q["iters"], R["iters"])
    assert np.array_equal(q["sigma"], R["sigma"])


def test_diverging_uneven_networks_converge():
    """The four networks of the 1024-network workload whose constant-step
    solves diverge (a fiber crushed and then stretched beyond the step's
    headroom): with the per-pass step (in groups of 16 workgroups, as the
    benchmark re-solves them) all converge, to the oracle's stress (bar:
    1e-8, or 100x the oracle's own spread over perturbed starts)."""
    path = os.path.join(GOLDEN, "uneven1024_steprule.json")
    if not os.path.exists(path):
        pytest.skip("the oracle's results for these networks (make_oracle_golden.py uneven_steprule) "
                    "are not stored")
    with open(path) as f:
        G = json.load(f)
    ids = [e["index"] for e in G["networks"]]
    sub = I.config_uneven_batch(1024, idx=ids)
    kw = dict(tol=1e-8, damping=G["damping"])
    r0 = solve(sub, tol=1e-8, max_iter=5000, damping=G["damping"])
    assert (r0["result"] == dr.DR_NONFINITE).all()
    g = solve(sub, dt_rule=1, tail_group=16, **kw)
    for k, e in enumerate(G["networks"]):
        o = e["tol_1e-08"]["plain"]
        s0 = np.array(o["sigma"])
        spread = max(rel(np.array(q["sigma"]), s0) for q in e["tol_1e-08"]["perturbed"])
        bar = max(1e-8, 100 * spread)
        err = rel(g["sigma"][k].ravel(), s0)
        # the oracle's residual and stress at the state the GPU returned
        crho, cs, _ = O.evaluate(sub.nets[k], sub.F[k], g["u_list"][k])
        say(f"net {e['index']} N={e['n_nodes']}: passes GPU {int(g['iters'][k])}, oracle {o['iters']}, "
            f"sigma rel {err:.2e} (bar {bar:.1e}); oracle residual at the GPU's state {crho:.2e}, "
            f"its stress there {rel(g['sigma'][k], cs):.1e}")
        assert o["status"] == O.CONVERGED and g["result"][k] == dr.DR_CONVERGED
        assert crho <= 1e-8 * (1 + 1e-6) and rel(g["sigma"][k], cs) < 1e-10
        assert err < bar


@pytest.mark.parametrize("group", [2, 4, 16])
def test_group_form_same_bits(group):
    """Every problem in a group of `group` workgroups from the start: at a
    fixed pass count the same bits as one workgroup per problem (the step
    bound is a max, exact in any order; sizes from one row per wave of the
    group to several), also across budgeted launches."""
    rng = np.random.default_rng(93)
    nets = [I.draw_network(rng, n) for n in (300, 2600, 9000, 21000)]
    base = I.Batch(nets, np.stack([np.diag([1.3, 1.0, 1.0])] * len(nets)))
    K = 1500
    kw = dict(tol=1e-300, max_iter=K, damping=1e-3, dt_rule=1)
    ref = solve(base, start=dr.DR_START_ZERO, **kw)
    got = solve(base, start=dr.DR_START_ZERO, tail_group=group, **kw)
    say(f"group {group}: passes {got['iters'].tolist()}, results {got['result'].tolist()}")
    assert np.array_equal(got["iters"], ref["iters"])
    assert np.array_equal(got["result"], ref["result"])
    assert np.array_equal(got["u"], ref["u"])
    assert np.array_equal(got["sigma"], ref["sigma"])
    # the same passes in budgeted group launches
    ids = np.arange(len(base), dtype=np.int32)
    b = dr.DRBatch(base, dt_safety=S, tail_group=group, **kw)
    b.advance(ids, np.full(len(ids), dr.DR_START_ZERO, np.int32), 400, F=base.F)
    for _ in range(10):
        run = ids[b.query(ids)["result"] == dr.DR_RUNNING]
        if len(run) == 0:
            break
        b.advance(run, np.full(len(run), dr.DR_RESUME, np.int32), 400)
    q = b.query(ids)
    b.close()
    assert np.array_equal(q["iters"], ref["iters"])
    assert np.array_equal(q["result"], ref["result"])
    assert np.array_equal(q["sigma"], ref["sigma"])


def test_group_form_converges_like_one_workgroup():
    """To convergence the group sums the norms in member order, so its stop
    pass may differ by one from one workgroup's; the stresses agree."""
    batch = stretched_batch()
    kw = dict(tol=1e-8, damping=1e-3, dt_rule=1)
    ref = solve(batch, start=dr.DR_START_ZERO, **kw)
    got = solve(batch, start=dr.DR_START_ZERO, tail_group=4, **kw)
    say("passes", got["iters"].tolist(), "one workgroup", ref["iters"].tolist())
    assert (got["result"] == dr.DR_CONVERGED).all()
    assert np.abs(got["iters"].astype(np.int64) - ref["iters"]).max() <= 1
    for i in range(len(batch)):
        assert rel(got["sigma"][i], ref["sigma"][i]) < 1e-9
