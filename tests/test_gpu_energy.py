"""Energy balance (Fig. 1, the optional check) on the GPU: the tracked work
terms against the oracle's, the balance itself, the guard, and that
tracking leaves the iteration unchanged."""
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


def oracle_all(batch, **kw):
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(lambda i: O.solve(batch.nets[i], batch.F[i], dt_safety=S, **kw),
                           range(len(batch))))


@pytest.mark.parametrize("placement", [dr.DR_PLACE_LDS, dr.DR_PLACE_GLOBAL])
def test_work_terms_match_oracle(placement):
    batch = I.small_batch(5, 90, 600, 0.02, seed=81)
    K = 300
    b = dr.DRBatch(batch, tol=1e-30, max_iter=K, damping=1e-3, dt_safety=S, placement=placement,
                   energy_tol=1.0)
    b.solve()
    g = b.results()
    e = b.energy()
    o = oracle_all(batch, tol=1e-30, max_iter=K, beta=1e-3)
    for i in range(len(batch)):
        say(f"net {i}: W {e['work_int'][i]:.12e} (oracle {o[i].work_int:.12e}), D {e['work_damp'][i]:.6e} "
            f"({o[i].work_damp:.6e}), KE {g['ke'][i]:.6e} ({o[i].ke:.6e})")
        assert g["result"][i] == dr.DR_MAX_ITER
        assert e["work_int"][i] == pytest.approx(o[i].work_int, rel=1e-8)
        assert e["work_damp"][i] == pytest.approx(o[i].work_damp, rel=1e-8)


def test_balance_and_tracking_leaves_iteration_unchanged():
    batch = I.small_batch(4, 100, 400, 0.02, seed=82)
    plain = dr.DRBatch(batch, tol=1e-8, damping=1e-3, dt_safety=S)
    plain.solve()
    p = plain.results()
    b = dr.DRBatch(batch, tol=1e-8, damping=1e-3, dt_safety=S, energy_tol=0.1)
    b.solve()
    g = b.results()
    e = b.energy()
    assert (g["result"] == dr.DR_CONVERGED).all()
    assert np.array_equal(g["sigma"], p["sigma"]) and np.array_equal(g["iters"], p["iters"])
    for i in range(len(batch)):
        W, D, KE = e["work_int"][i], e["work_damp"][i], g["ke"][i]
        bal = abs(KE - W + D) / max(KE, abs(W), D)
        say(f"net {i}: W {W:.6e} D {D:.6e} KE {KE:.2e} balance {bal:.2e}")
        assert W > 0 and D > 0 and bal < 3e-3


def test_guard_trips_at_first_check_and_chunked_equals_single():
    batch = I.small_batch(3, 100, 300, 0.02, seed=83)
    # a tolerance no explicit step meets: the solve ends at the first check
    b = dr.DRBatch(batch, tol=1e-8, damping=1e-3, dt_safety=S, energy_tol=1e-12)
    b.solve()
    g = b.results()
    say("guard:", list(g["result"]), list(g["iters"]))
    assert (g["result"] == dr.DR_ENERGY).all() and (g["iters"] == 1024).all()
    # the tracked terms survive budgeted launches exactly
    one = dr.DRBatch(batch, tol=1e-8, damping=1e-3, dt_safety=S, energy_tol=0.1)
    one.solve()
    r1, e1 = one.results(), one.energy()
    ch = dr.DRBatch(batch, tol=1e-8, damping=1e-3, dt_safety=S, energy_tol=0.1)
    ids = np.arange(len(batch), dtype=np.int32)
    ch.advance(ids, [dr.DR_START_AFFINE] * len(ids), 3333, F=batch.F)
    for _ in range(1000):
        q = ch.query(ids)
        run = ids[q["result"] == dr.DR_RUNNING]
        if len(run) == 0:
            break
        ch.advance(run, [dr.DR_RESUME] * len(run), 3333)
    e2 = ch.energy()
    assert np.array_equal(q["sigma"], r1["sigma"]) and np.array_equal(q["iters"], r1["iters"])
    assert np.array_equal(e2["work_int"], e1["work_int"])
    assert np.array_equal(e2["work_damp"], e1["work_damp"])
    with pytest.raises(dr.DrError):
        dr.DRBatch(batch, tol=1e-8).energy()
