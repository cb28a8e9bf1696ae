"""Macroscale tangent by warm-started perturbation solves (the FE2 step of
section I after the stress): on the cubic lattice against the derivative of
its closed-form stress, on kNN networks against the oracle running the same
sequence of warm-started solves."""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as O
from paper_2305_07030_amd import dr
from paper_2305_07030_amd import inputs as I
from paper_2305_07030_amd import tangent as TG

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


def lattice_sigma(F, m, EA):
    J = np.linalg.det(F)
    return sum((m + 1) ** 2 / J * EA * (np.linalg.norm(F[:, k]) ** 2 - 1) / (2 * np.linalg.norm(F[:, k]))
               * np.outer(F[:, k], F[:, k]) for k in range(3))


def test_lattice_tangent_closed_form():
    m, EA, h = 3, 1.3, 1e-3
    lat = I.cubic_lattice(m, EA=EA)
    F = np.array([[1.05, 0.02, 0.0], [0.02, 1.03, 0.01], [0.0, 0.01, 1.04]])
    b = dr.DRBatch(I.Batch([lat], F[None]), tol=1e-12, damping=0.02)
    t = TG.tangent(b, F[None], h=h)
    assert (t["results"] == dr.DR_CONVERGED).all()
    D = t["D"][0]
    ref = np.zeros((3, 3, 3, 3))
    for k, l in TG.DIRECTIONS:
        E = TG.sym_dir(k, l)
        d = (lattice_sigma(F + h * E, m, EA) - lattice_sigma(F - h * E, m, EA)) / (2 * h)
        ref[:, :, k, l] = d
        ref[:, :, l, k] = d
    err = np.linalg.norm(D - ref) / np.linalg.norm(ref)
    say(f"lattice tangent rel err {err:.2e}, passes {int(t['passes'][0])}")
    assert err < 1e-9
    assert np.allclose(t["sigma"][0], lattice_sigma(F, m, EA), rtol=1e-10, atol=0)


def oracle_tangent(net, F, h, tol, beta):
    r = O.solve(net, F, tol=tol, beta=beta, dt_safety=0.9)
    sig0, u, Fp = r.sigma, r.u, F
    D = np.zeros((3, 3, 3, 3))
    for k, l in TG.DIRECTIONS:
        E = TG.sym_dir(k, l)
        s = []
        for sgn in (1.0, -1.0):
            Fn = F + sgn * h * E
            r = O.solve(net, Fn, tol=tol, beta=beta, dt_safety=0.9, start=O.START_WARM, F_prev=Fp, u_prev=u)
            s.append(r.sigma)
            u, Fp = r.u, Fn
        D[:, :, k, l] = D[:, :, l, k] = (s[0] - s[1]) / (2 * h)
    return sig0, D


def test_knn_tangent_against_oracle():
    batch = I.small_batch(4, 100, 250, 0.02, seed=73)
    tol, beta, h = 1e-10, 1e-3, 1e-3
    b = dr.DRBatch(batch, tol=tol, damping=beta, dt_safety=0.9)
    t = TG.tangent(b, batch.F, h=h)
    assert (t["results"] == dr.DR_CONVERGED).all()
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        ref = list(ex.map(lambda i: oracle_tangent(batch.nets[i], batch.F[i], h, tol, beta),
                          range(len(batch))))
    for i, (s0, D) in enumerate(ref):
        err = np.linalg.norm(t["D"][i] - D) / np.linalg.norm(D)
        say(f"net {i}: tangent rel err {err:.2e}, passes {int(t['passes'][i])}")
        assert err < 1e-5
        assert np.linalg.norm(t["sigma"][i] - s0) < 1e-8 * np.linalg.norm(s0)
