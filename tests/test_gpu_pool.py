"""The library's serving pool (dr_pool_*): every request's result equals,
bit for bit, a plain warm-started solve of the same sequence of F's of its
network; requests of one network are served in order; the caps hold."""
import sys

import numpy as np
import pytest

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


def test_pool_matches_sequential_warm_solves():
    batch = I.small_batch(6, 80, 900, 0.02, seed=95)
    rng = np.random.default_rng(96)
    kw = dict(tol=1e-8, damping=1e-3, dt_safety=S)
    # 3 requests per network, F walking by symmetric steps, interleaved
    reqs = []
    F = batch.F.copy()
    for rnd in range(3):
        for p in rng.permutation(len(batch)):
            e = rng.uniform(-0.003, 0.003, 6)
            F[p] = F[p] + np.array([[e[0], e[1], e[2]], [e[1], e[3], e[4]], [e[2], e[4], e[5]]])
            reqs.append((int(p), F[p].copy()))
    nodes = np.array([n.n_nodes for n in batch.nets])
    budget = int(dr.state_bytes_per_node() * np.sort(nodes)[-3:].sum())  # about three of the largest in flight
    pool = dr.Pool(batch, state_budget_bytes=budget, max_slots=4, tick_passes=300, **kw)
    for tag, (p, Fp) in enumerate(reqs):
        pool.submit(p, Fp, tag)
    got = {}
    order = []
    for tick in range(100000):
        st = pool.status()
        assert st["in_flight"] <= 4 and st["state_bytes"] <= budget
        out = pool.poll(max_out=2)
        for t, i, sg, r, it in zip(out["tags"], out["ids"], out["sigma"], out["result"], out["iters"]):
            got[int(t)] = (int(i), sg.copy(), int(r), int(it))
            order.append(int(t))
        st = pool.status()
        if st["queued"] == 0 and st["in_flight"] == 0 and st["completed"] == 0:
            break
    say(f"{len(got)} results after {tick + 1} polls")
    assert sorted(got) == list(range(len(reqs)))
    # per network, results come out in submission order
    for p in range(len(batch)):
        tags = [t for t in order if got[t][0] == p]
        assert tags == sorted(tags)
    # reference: the same F sequence per network, plain warm-started solves
    ref = dr.DRBatch(batch, **kw)
    for tag, (p, Fp) in enumerate(reqs):
        ref.solve(F=Fp[None], ids=np.array([p], np.int32), start=dr.DR_START_WARM)
        r = ref.results()
        i, sg, res, it = got[tag]
        assert i == p and res == dr.DR_CONVERGED
        assert it == int(r["iters"][0]), (tag, it, int(r["iters"][0]))
        assert np.array_equal(sg, r["sigma"][0]), tag
    ref.close()
    pool.close()


def test_pool_rejections():
    batch = I.small_batch(2, 60, 200, 0.02, seed=97)
    pool = dr.Pool(batch, state_budget_bytes=dr.state_bytes_per_node() * 10, max_slots=1, tick_passes=100)
    with pytest.raises(dr.DrError):  # the network alone is over the budget
        pool.submit(0, np.eye(3), 0)
    with pytest.raises(dr.DrError):
        pool.submit(5, np.eye(3), 0)
    with pytest.raises(dr.DrError):
        pool.submit(0, -np.eye(3), 0)
    out = pool.poll()
    assert len(out["tags"]) == 0
    pool.close()


def test_advance_each_budgets():
    """dr_advance_each: slot k makes exactly its own budget of passes; the
    solves then resumed to a fixed total pass count give the same bits as one
    launch (each problem's arithmetic does not depend on its budget)."""
    batch = I.small_batch(4, 100, 2000, 0.02, seed=97)
    K = 5000
    kw = dict(tol=1e-300, max_iter=K, damping=1e-3, dt_safety=S)
    ref = dr.DRBatch(batch, **kw)
    ref.solve()
    R = ref.results()
    ref.close()
    ids = np.arange(len(batch), dtype=np.int32)
    b = dr.DRBatch(batch, **kw)
    budgets = np.array([100, 250, 1000, 3000], np.int64)
    b.advance(ids, np.full(len(ids), dr.DR_START_AFFINE, np.int32), budgets, F=batch.F)
    q = b.query(ids)
    say("after one launch:", q["iters"].tolist())
    assert np.array_equal(q["iters"], budgets) and (q["result"] == dr.DR_RUNNING).all()
    costs = b.pass_costs()
    assert (costs > 0).all() and costs[np.argmax([n.n_fibers for n in batch.nets])] == costs.max()
    for _ in range(100):
        run = ids[b.query(ids)["result"] == dr.DR_RUNNING]
        if len(run) == 0:
            break
        b.advance(run, np.full(len(run), dr.DR_RESUME, np.int32), np.full(len(run), 700, np.int64))
    q = b.query(ids)
    b.close()
    assert (q["result"] == dr.DR_MAX_ITER).all() and (q["iters"] == K).all()
    assert np.array_equal(q["sigma"], R["sigma"])
