"""Chunked (resumable) solves and the FP32-state path, through the C ABI.

* A solve split over several budgeted launches (dr_advance) must give the
  same bits as one dr_solve: the saved state is exact and each problem's
  arithmetic is independent of the other slots of a launch.
* FP32 nodal state and force gather, FP64 norms and stress: checked against
  the FP64 oracle within a stated bound, and exactly zero where the Green
  strain form makes it exact.
"""
import os
import sys
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


@pytest.mark.parametrize("placement", [dr.DR_PLACE_LDS, dr.DR_PLACE_GLOBAL])
def test_chunked_equals_single_launch(placement):
    batch = I.small_batch(9, 80, 600, 0.02, seed=31)
    say(f"chunked vs single launch, placement {placement}, N =", [n.n_nodes for n in batch.nets])
    one = dr.DRBatch(batch, tol=1e-8, damping=1e-3, dt_safety=S, placement=placement)
    one.solve()
    ref = one.results(want_u=True)
    ch = dr.DRBatch(batch, tol=1e-8, damping=1e-3, dt_safety=S, placement=placement)
    ids = np.arange(len(batch), dtype=np.int32)
    assert (ch.query(ids)["result"] == dr.DR_IDLE).all()
    ch.advance(ids, np.full(len(ids), dr.DR_START_AFFINE, np.int32), 3000, F=batch.F)
    launches = 1
    while True:
        q = ch.query(ids)
        running = ids[q["result"] == dr.DR_RUNNING]
        if len(running) == 0:
            break
        ch.advance(running, np.full(len(running), dr.DR_RESUME, np.int32), 3000)
        launches += 1
        assert launches < 1000
    say("launches", launches, "passes", list(q["iters"]))
    assert launches > 2
    assert np.array_equal(q["iters"], ref["iters"])
    assert np.array_equal(q["sigma"], ref["sigma"])
    assert np.array_equal(q["sigma_fib"], ref["sigma_fib"])
    assert np.array_equal(q["result"], ref["result"])
    u_ch = dr.dr_stress(ch.h, len(ids), ch.total_nodes, True)["u"]
    assert np.array_equal(u_ch, ref["u"])


@pytest.mark.parametrize("precision", [dr.DR_FP64, dr.DR_FP32])
def test_resume_across_placements(precision):
    """A running solve saved by one placement resumes under the other (the
    class plans change between launches, odd and even budgets so both state
    buffers serve as the saved one): the same bits as one launch."""
    batch = I.small_batch(6, 80, 500, 0.02, seed=34)
    kw = dict(tol=1e-8 if precision == dr.DR_FP64 else 1e-6, damping=1e-3, dt_safety=S,
              precision=precision, stall_window=50000 if precision == dr.DR_FP32 else 0)
    one = dr.DRBatch(batch, **kw)
    one.solve()
    ref = one.results()
    ch = dr.DRBatch(batch, **kw)
    ids = np.arange(len(batch), dtype=np.int32)
    plans = [[dict(n_hi=100000, block=512, chunk=1, placement=dr.DR_PLACE_LDS)],
             [dict(n_hi=100000, block=1024, chunk=1, placement=dr.DR_PLACE_GLOBAL)]]
    ch.set_class_plans(plans[0])
    ch.advance(ids, np.full(len(ids), dr.DR_START_AFFINE, np.int32), 2999, F=batch.F)
    k = 1
    while True:
        q = ch.query(ids)
        running = ids[q["result"] == dr.DR_RUNNING]
        if len(running) == 0:
            break
        ch.set_class_plans(plans[k % 2])
        ch.advance(running, np.full(len(running), dr.DR_RESUME, np.int32), 2999 + (k % 2))
        k += 1
        assert k < 1000
    say(f"precision {precision}: {k} launches, passes {list(q['iters'])}")
    assert k > 3
    assert np.array_equal(q["iters"], ref["iters"])
    assert np.array_equal(q["sigma"], ref["sigma"])
    assert np.array_equal(q["result"], ref["result"])
    one.close()
    ch.close()


def test_mixed_fresh_and_resumed_slots():
    """A launch may start some problems and resume others; results equal the
    same solves run alone."""
    batch = I.small_batch(6, 100, 400, 0.02, seed=32)
    b = dr.DRBatch(batch, tol=1e-8, damping=1e-3, dt_safety=S)
    alone = dr.DRBatch(batch, tol=1e-8, damping=1e-3, dt_safety=S)
    alone.solve()
    ref = alone.results()
    say("mixed slots")
    b.advance([0, 1, 2], [dr.DR_START_AFFINE] * 3, 500, F=batch.F[:3])
    b.advance([0, 1, 2, 3, 4, 5], [dr.DR_RESUME] * 3 + [dr.DR_START_AFFINE] * 3, 700,
              F=np.concatenate([np.tile(np.eye(3), (3, 1, 1)), batch.F[3:]]))
    ids = np.arange(6, dtype=np.int32)
    for _ in range(1000):
        q = b.query(ids)
        run = ids[q["result"] == dr.DR_RUNNING]
        if len(run) == 0:
            break
        b.advance(run, [dr.DR_RESUME] * len(run), 2000)
    assert np.array_equal(q["sigma"], ref["sigma"]) and np.array_equal(q["iters"], ref["iters"])


def test_resume_of_finished_solve_rejected_or_noop():
    batch = I.small_batch(2, 60, 80, 0.02, seed=33)
    b = dr.DRBatch(batch, tol=1e-8, damping=1e-3, dt_safety=S)
    with pytest.raises(dr.DrError):
        b.advance([0], [dr.DR_RESUME], 10)  # never started
    b.advance([0, 1], [dr.DR_START_AFFINE] * 2, 10 ** 7, F=batch.F)
    q = b.query(np.array([0, 1], np.int32))
    assert (q["result"] == dr.DR_CONVERGED).all()
    with pytest.raises(dr.DrError):
        b.advance([0], [dr.DR_RESUME], 10)  # finished


def oracle_all(batch, **kw):
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(lambda i: O.solve(batch.nets[i], batch.F[i], dt_safety=S, **kw),
                           range(len(batch))))


FP32_SIGMA_BOUND = 2e-3  # stated bound of the FP32 path against the FP64 oracle
FP32_STALL = 50_000


def test_fp32_against_fp64_oracle():
    """FP32 force rounding (~1e-7 relative per fiber force, a floor near
    1e-6 under rho) is re-injected every pass and integrated by the lightly
    damped high-frequency modes (damping ratio ~beta/2), which amplify it by
    ~1/sqrt(beta/2) ~ 45: the residual then wanders near 1e-5..1e-4.  A solve
    ends converged or stalled (no 0.1 % progress in 50 000 passes); the
    reached residual is reported (within 1e-3 here), and the stress is within
    the stated bound."""
    batch = I.small_batch(10, 100, 700, 0.02, seed=34)
    say("FP32 state, tol 1e-6, N =", [n.n_nodes for n in batch.nets])
    b = dr.DRBatch(batch, tol=1e-6, damping=1e-3, dt_safety=S, precision=dr.DR_FP32,
                   stall_window=FP32_STALL)
    b.solve()
    g = b.results(want_u=True)
    o = oracle_all(batch, tol=1e-8, beta=1e-3)
    errs = [rel(g["sigma"][i], o[i].sigma) for i in range(len(batch))]
    say("FP32 sigma rel err vs FP64 oracle:", ["%.1e" % e for e in errs],
        "passes", list(g["iters"]), "oracle", [x.iters for x in o],
        "status", list(g["result"]), "rho", ["%.1e" % x for x in g["rho"]])
    assert np.isin(g["result"], [dr.DR_CONVERGED, dr.DR_STALLED]).all()
    assert (g["rho"] <= 1e-3).all()
    assert max(errs) < FP32_SIGMA_BOUND
    # FP32 run-to-run repeatability
    b.solve()
    g2 = b.results()
    assert np.array_equal(g2["sigma"], g["sigma"])


def test_fp32_closed_forms():
    say("FP32 closed forms: identity is exactly zero; lattice from u = 0")
    base = I.config_single(200, seed=3).nets[0]
    b = dr.DRBatch(I.Batch([base], np.eye(3)[None]), tol=1e-6, precision=dr.DR_FP32)
    b.solve()
    g = b.results(want_u=True)
    assert g["iters"][0] == 1 and np.array_equal(g["sigma"][0], np.zeros((3, 3)))
    assert np.array_equal(g["u"], np.zeros_like(g["u"]))
    m = 3
    lat = I.cubic_lattice(m, EA=1.3)
    F = np.array([[1.05, 0.02, 0.0], [0.01, 1.03, 0.0], [0.0, 0.015, 1.04]])
    b = dr.DRBatch(I.Batch([lat], F[None]), tol=1e-6, damping=0.02, precision=dr.DR_FP32,
                   stall_window=FP32_STALL)
    b.solve(start=dr.DR_START_ZERO)
    g = b.results(want_u=True)
    J = np.linalg.det(F)
    sig = sum((m + 1) ** 2 / J * 1.3 * (np.linalg.norm(F[:, k]) ** 2 - 1) / (2 * np.linalg.norm(F[:, k]))
              * np.outer(F[:, k], F[:, k]) for k in range(3))
    assert g["result"][0] == dr.DR_CONVERGED
    assert np.abs(g["u"] - lat.X @ (F - np.eye(3)).T).max() < 1e-5
    assert rel(g["sigma"][0], sig) < 1e-4


def test_fp32_chunked_equals_single():
    batch = I.small_batch(4, 150, 500, 0.02, seed=35)
    """Chunked FP32 solves, including the stall guard's progress carried
    across launches, give the bits of one launch."""
    one = dr.DRBatch(batch, tol=1e-6, damping=1e-3, dt_safety=S, precision=dr.DR_FP32,
                     stall_window=FP32_STALL)
    one.solve()
    ref = one.results()
    ch = dr.DRBatch(batch, tol=1e-6, damping=1e-3, dt_safety=S, precision=dr.DR_FP32,
                    stall_window=FP32_STALL)
    ids = np.arange(len(batch), dtype=np.int32)
    ch.advance(ids, [dr.DR_START_AFFINE] * len(ids), 17_777, F=batch.F)
    for _ in range(1000):
        q = ch.query(ids)
        run = ids[q["result"] == dr.DR_RUNNING]
        if len(run) == 0:
            break
        ch.advance(run, [dr.DR_RESUME] * len(run), 17_777)
    say("FP32 chunked: status", list(q["result"]), "passes", list(q["iters"]))
    assert np.array_equal(q["result"], ref["result"])
    assert np.array_equal(q["sigma"], ref["sigma"]) and np.array_equal(q["iters"], ref["iters"])


def test_fp32_uniform_batch_against_oracle():
    """The 256-network workload with FP32 state (the benchmark's FP32
    configuration: damping 3e-2, tol 1e-6, stall guard 50 000 passes), against
    the FP64 oracle on the stratified sample of 16 networks stored in
    tests/golden/uniform256_sample.json (the oracle's solves at tol 1e-10).
    Per network: the stress error against the oracle, the FP64 residual of
    the FP32 state by the oracle's own definition (rho64), and the oracle's
    own spread over 1e-15-perturbed starts.  Stated bound: where the oracle's
    equilibrium is stable (spread below 1e-7) the stress error is at most
    500 max(rho64, 1e-6) (the stress of a state moves with its residual;
    observed factors 1.6-200 on this sample, stress errors 1.6e-6 to
    4.3e-3); every FP32 state has rho64 below 1e-3; its stress is the FP64
    stress of that state."""
    import json
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "uniform256_sample.json")) as f:
        G = json.load(f)
    batch = I.config_uniform_batch(256)
    b = dr.DRBatch(batch, tol=1e-6, damping=3e-2, dt_safety=S, precision=dr.DR_FP32,
                   stall_window=FP32_STALL)
    b.solve()
    g = b.results(want_u=True)
    b.close()
    say("FP32 batch: converged", int((g["result"] == dr.DR_CONVERGED).sum()), "stalled",
        int((g["result"] == dr.DR_STALLED).sum()), "rho median", float(np.median(g["rho"])))
    errs = []
    for e in G["networks"]:
        i = e["index"]
        o = e["tol_1e-10"]["plain"]
        if o["status"] != O.CONVERGED:
            o = e["tol_1e-08"]["plain"]
        s0 = np.array(o["sigma"]).reshape(3, 3)
        err = rel(g["sigma"][i], s0)
        rho64, s64, _ = O.evaluate(batch.nets[i], batch.F[i], g["u_list"][i])
        spread = max(rel(np.array(q["sigma"]).reshape(3, 3), s0) for q in e["tol_1e-08"]["perturbed"])
        say(f"net {i:3d} N={e['n_nodes']} ({e['why']}): FP32 status {int(g['result'][i])} passes "
            f"{int(g['iters'][i])} rho {g['rho'][i]:.1e}; FP64 residual of its state {rho64:.1e}; sigma rel "
            f"err vs oracle {err:.1e} (oracle spread at tol 1e-8 {spread:.1e})")
        errs.append((i, int(g["result"][i]), err, spread, rho64, rel(g["sigma"][i], s64)))
    e = np.array([x[2] for x in errs])
    say(f"sigma rel err vs oracle: median {np.median(e):.1e}, p90 {np.percentile(e, 90):.1e}, max {e.max():.1e}")
    ratio = [x[2] / max(x[4], 1e-6) for x in errs if x[3] < 1e-7]
    say(f"stable-equilibrium networks: sigma error / max(rho64, 1e-6) up to {max(ratio):.1f}")
    for i, st, err, spread, rho64, cs in errs:
        assert st in (dr.DR_CONVERGED, dr.DR_STALLED, dr.DR_MAX_ITER)
        assert rho64 < 1e-3
        assert cs < 1e-10  # the stress of the state, in FP64
        if spread < 1e-7:
            assert err < 500 * max(rho64, 1e-6), (i, err, rho64)
