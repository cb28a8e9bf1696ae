"""Running-state records and network input rules, through the C ABI: a
launch-loop solve leaves the saved state of another problem's running solve
alone; the band rule (fixed = NULL) gives the same solve as the explicit
mask."""
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


@pytest.mark.parametrize("placement", [dr.DR_PLACE_LDS, dr.DR_PLACE_GLOBAL])
def test_loop_solve_keeps_other_running_state(placement):
    """Problem 1 is advanced by a budget and left running; problem 0 is then
    solved by the launch loop; problem 1 resumes and must give the same bits
    as one uninterrupted solve."""
    batch = I.small_batch(2, 300, 500, 0.02, seed=31)
    kw = dict(tol=1e-8, damping=1e-3, dt_safety=S, placement=placement)
    say("loop solve between the launches of a running solve, N =", [n.n_nodes for n in batch.nets],
        "placement", placement)
    ref = dr.DRBatch(batch, **kw)
    ref.solve()
    R = ref.results(want_u=True)
    ref.close()
    b = dr.DRBatch(batch, **kw)
    ids = np.array([0, 1], np.int32)
    b.advance(ids, np.full(2, dr.DR_START_AFFINE, np.int32), 500, F=batch.F)
    q = b.query(ids)
    assert (q["result"] == dr.DR_RUNNING).all()
    b.solve_loop(F=batch.F[[0]], ids=np.array([0], np.int32))
    L = b.results()
    assert L["result"][0] == dr.DR_CONVERGED
    b.advance(np.array([1], np.int32), np.array([dr.DR_RESUME], np.int32), 10 ** 7)
    q = b.query(np.array([1], np.int32))
    say("resumed problem 1:", int(q["iters"][0]), "passes, uninterrupted", int(R["iters"][1]))
    assert q["result"][0] == dr.DR_CONVERGED
    assert q["iters"][0] == R["iters"][1]
    assert np.array_equal(q["sigma"][0], R["sigma"][1])
    b.close()


def test_band_rule_equals_explicit_mask():
    batch = I.small_batch(3, 200, 600, 0.02, seed=32)
    say("band rule vs explicit prescribed mask, N =", [n.n_nodes for n in batch.nets])
    pk = batch.packed()
    opt = dr.make_options(tol=1e-8, damping=1e-3, dt_safety=S)
    outs = []
    for p in (pk, dict(pk, fixed=None, band=I.BAND)):
        h = dr.dr_batch_create(p, opt, dr.current_stream())
        dr.dr_solve(h, batch.F)
        outs.append(dr.dr_stress(h, len(batch)))
        dr.dr_batch_destroy(h)
    assert (outs[0]["result"] == dr.DR_CONVERGED).all()
    assert np.array_equal(outs[0]["sigma"], outs[1]["sigma"])
    assert np.array_equal(outs[0]["iters"], outs[1]["iters"])
