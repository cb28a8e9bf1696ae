"""Pins of the CPU oracle against facts the oracle does not compute itself.

Each test states the passage of the paper (or the reading of it) that fixes
the expected value.  Together they are chosen so that a plausible mistake in
the oracle (a dropped factor, a wrong sign or index, a transposed operand, a
wrong time-integration coefficient) fails at least one of them.
"""
import math

import numpy as np
import pytest

from paper_2305_07030_amd import inputs as I

BETA = 1e-3
S = 0.9


def _net(X, fibers, EA, fixed):
    return I.Network(np.asarray(X, float), np.asarray(fibers, np.int32), np.asarray(EA, float),
                     np.asarray(fixed, np.uint8))


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


# --------------------------------------------------------------------------
# P1: one fiber with both ends prescribed -- force law and stress average
# (fiber law reading T = EA (lambda^2 - 1) / 2; stress as the boundary average)
# --------------------------------------------------------------------------
def test_single_fiber_closed_form(oracle_lib):
    O = oracle_lib
    X = [[0.2, 0.3, 0.4], [0.7, 0.6, 0.5]]
    EA = 1.7
    net = _net(X, [[0, 1]], [EA], [1, 1])
    F = np.array([[1.1, 0.05, 0.0], [0.02, 0.95, 0.03], [0.0, 0.01, 1.02]])
    r = O.solve(net, F, tol=1e-8, beta=BETA, dt_safety=S)
    x = np.asarray(X) @ F.T
    d = x[1] - x[0]
    l = np.linalg.norm(d)
    L = np.linalg.norm(np.subtract(X[1], X[0]))
    T = EA * ((l / L) ** 2 - 1) / 2
    sig = T * np.outer(d, d) / l / np.linalg.det(F)
    assert r.status == O.CONVERGED and r.iters == 1  # repeat-until: one pass
    assert np.allclose(r.u, np.asarray(X) @ (F - np.eye(3)).T, rtol=0, atol=1e-15)
    assert _rel(r.sigma, sig) < 1e-13
    assert _rel(r.sigma_fib, sig) < 1e-13


# --------------------------------------------------------------------------
# P2: collinear two-fiber chain, middle node free -- equilibrium by bisection
# --------------------------------------------------------------------------
def _chain():
    X = [[0.2, 0.5, 0.5], [0.45, 0.5, 0.5], [0.8, 0.5, 0.5]]
    return _net(X, [[0, 1], [1, 2]], [1.0, 1.7], [1, 0, 1])


def _chain_equilibrium(net, F):
    L1, L2 = 0.25, 0.35
    EA1, EA2 = net.EA
    xA, xC = F @ net.X[0], F @ net.X[2]
    ell = np.linalg.norm(xC - xA)
    e = (xC - xA) / ell

    def h(l1):  # tension in fiber 1 minus tension in fiber 2
        l2 = ell - l1
        return EA1 * ((l1 / L1) ** 2 - 1) / 2 - EA2 * ((l2 / L2) ** 2 - 1) / 2

    lo, hi = 1e-9, ell - 1e-9
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if h(mid) > 0:
            hi = mid
        else:
            lo = mid
    l1 = 0.5 * (lo + hi)
    T = EA1 * ((l1 / L1) ** 2 - 1) / 2
    xB = xA + l1 * e
    return xB, T, ell, e


def test_chain_equilibrium_bisection(oracle_lib):
    O = oracle_lib
    net = _chain()
    F = np.diag([1.05, 1.0, 1.0])
    r = O.solve(net, F, tol=1e-12, beta=0.05, dt_safety=S)
    xB, T, ell, e = _chain_equilibrium(net, F)
    assert r.status == O.CONVERGED
    assert np.allclose(net.X[1] + r.u[1], xB, rtol=0, atol=1e-12)
    sig = T * ell * np.outer(e, e) / np.linalg.det(F)
    assert _rel(r.sigma, sig) < 1e-10
    assert _rel(r.sigma_fib, sig) < 1e-10


def test_chain_linear_trajectory(oracle_lib):
    """Integrator pin: near equilibrium the chain is a 1-DOF damped oscillator
    with omega^2 = (EA1 lam1 / L1 + EA2 lam2 / L2) / m_B (tangent of the fiber
    law).  Fig. 1's loop (half velocity update, displacement update, force,
    damping with the half-step velocity, acceleration, half velocity update)
    is then, on the offset u and the half-step velocity w,
        u_n = u_{n-1} + dt w_n,  w_{n+1} = (1 - c dt) w_n - dt omega^2 u_n,
    started from u_0 = delta, w_1 = -(dt / 2) omega^2 delta.  The residual of
    pass n is proportional to |u_n|."""
    O = oracle_lib
    net = _chain()
    F = np.diag([1.05, 1.0, 1.0])
    xB, T, ell, e = _chain_equilibrium(net, F)
    L1, L2 = 0.25, 0.35
    l1 = np.linalg.norm(xB - F @ net.X[0]); l2 = ell - l1
    kt = net.EA[0] * (l1 / L1) / L1 + net.EA[1] * (l2 / L2) / L2
    mB = 0.5 * (L1 + L2)
    om2 = kt / mB
    delta = 1e-7
    u_prev = np.vstack([F @ x - x for x in net.X])
    u_prev[1] = xB - net.X[1] + delta * e
    K = 300
    r = O.solve(net, F, tol=1e-300, max_iter=K, beta=0.02, dt_safety=S,
                start=O.START_WARM, F_prev=F, u_prev=u_prev, trace_len=K)
    dt, c = r.dt, r.c
    u, w = delta, -0.5 * dt * om2 * delta
    pred = []
    for _ in range(K):
        u = u + dt * w
        pred.append(abs(u))
        w = (1 - c * dt) * w - dt * om2 * u
    pred = np.array(pred) / pred[0]
    got = r.rho_trace / r.rho_trace[0]
    assert np.abs(got - pred).max() < 1e-4, np.abs(got - pred).max()
    # and it decays at the spectral radius sqrt(1 - c dt) of the linear map
    assert pred[-50:].max() < 0.5 * pred[:50].max()


def test_stress_forms_identity_off_equilibrium(oracle_lib):
    """At any state: sigma - sigma_fib = 1/J sum_free g_i (x) (x_i - F c0),
    because sum over all nodes of g (x) (x - F c0) = -J sigma_fib."""
    O = oracle_lib
    b = I.config_single(200, seed=6)
    net = b.nets[0]
    F = I.sym_perturbed_F(np.random.default_rng(8), 0.02)
    r = O.solve(net, F, tol=1e-12, max_iter=3, beta=BETA, dt_safety=S, start=O.START_ZERO)
    assert r.status == O.MAX_ITER
    g = O.internal_force(net, r.u)
    x = net.X + r.u
    y = x - F @ np.full(3, 0.5)
    fr = net.fixed == 0
    rhs = (g[fr].T @ y[fr]) / np.linalg.det(F)
    assert np.linalg.norm(rhs) > 1e-3 * np.linalg.norm(r.sigma)  # far from equilibrium
    assert np.abs((r.sigma - r.sigma_fib) - rhs).max() < 1e-12 * np.abs(r.sigma).max()


# --------------------------------------------------------------------------
# P3: regular cubic lattice -- exact affine equilibrium and closed-form stress
# --------------------------------------------------------------------------
def test_lattice_affine_closed_form(oracle_lib):
    O = oracle_lib
    m = 3
    net = I.cubic_lattice(m, EA=1.3)
    assert net.n_fixed == (m + 1) ** 3 - (m - 1) ** 3
    F = np.array([[1.05, 0.02, 0.0], [0.01, 1.03, 0.0], [0.0, 0.015, 1.04]])
    r = O.solve(net, F, tol=1e-12, beta=0.02, dt_safety=S, start=O.START_ZERO)
    assert r.status == O.CONVERGED
    assert np.allclose(r.u, net.X @ (F - np.eye(3)).T, rtol=0, atol=1e-11)
    J = np.linalg.det(F)
    sig = np.zeros((3, 3))
    for k in range(3):
        Fe = F[:, k]
        lam = np.linalg.norm(Fe)
        sig += (m + 1) ** 2 / J * 1.3 * (lam ** 2 - 1) / (2 * lam) * np.outer(Fe, Fe)
    assert _rel(r.sigma, sig) < 1e-9
    assert _rel(r.sigma_fib, sig) < 1e-9
    # from the affine start the lattice is already in equilibrium
    r2 = O.solve(net, F, tol=1e-12, beta=0.02, dt_safety=S)
    assert r2.iters == 1 and _rel(r2.sigma, sig) < 1e-12


# --------------------------------------------------------------------------
# P4: rigid rotation carries no stress
# --------------------------------------------------------------------------
def test_rotation_zero_stress(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(11)
    R = I.random_rotation(rng)
    net = I.config_single(200, seed=3).nets[0]
    r = O.solve(net, R, tol=1e-8, beta=BETA, dt_safety=S)
    assert r.status == O.CONVERGED and r.iters == 1
    assert np.abs(r.sigma).max() < 1e-13
    # perturbed start on a rigid (complete) network relaxes back to sigma = 0
    cn = I.complete_network(rng, 8, 4)
    u0 = cn.X @ (R - np.eye(3)).T
    u0[4:] += rng.uniform(-0.01, 0.01, size=(4, 3))
    r = O.solve(cn, R, tol=1e-10, beta=0.05, dt_safety=S, start=O.START_WARM, F_prev=R, u_prev=u0)
    assert r.status == O.CONVERGED
    d = O.derived(cn, 0.05, S)
    assert np.abs(r.sigma).max() < 100 * 1e-10 * d["s_floor"]
    assert np.allclose(r.u, cn.X @ (R - np.eye(3)).T, atol=1e-8)


# --------------------------------------------------------------------------
# P5: objectivity -- F and R F give rotated trajectories
# --------------------------------------------------------------------------
def test_objectivity(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(5)
    net = I.config_single(120, seed=7).nets[0]
    F = I.sym_perturbed_F(rng, 0.02)
    R = I.random_rotation(rng)
    a = O.solve(net, F, tol=1e-9, beta=BETA, dt_safety=S)
    b = O.solve(net, R @ F, tol=1e-9, beta=BETA, dt_safety=S)
    assert a.status == b.status == O.CONVERGED
    assert abs(a.iters - b.iters) <= 1
    assert _rel(b.sigma, R @ a.sigma @ R.T) < 1e-8
    xa = net.X + a.u
    xb = net.X + b.u
    assert np.abs(xb - xa @ R.T).max() < 1e-8


# --------------------------------------------------------------------------
# P6: invariants of the internal force (any state) and of the converged stress
# --------------------------------------------------------------------------
def test_force_balance_invariants(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(2)
    net = I.config_single(300, seed=4).nets[0]
    u = rng.uniform(-0.03, 0.03, size=net.X.shape)
    g = O.internal_force(net, u)
    x = net.X + u
    scale = np.abs(g).max()
    assert np.abs(g.sum(0)).max() < 1e-12 * scale * net.n_nodes
    assert np.abs(np.cross(x, g).sum(0)).max() < 1e-12 * scale * net.n_nodes


def test_force_is_minus_energy_gradient(oracle_lib):
    """g = -dW/dx with W the integral of the fiber law (central differences)."""
    O = oracle_lib
    rng = np.random.default_rng(9)
    net = I.config_single(60, seed=1).nets[0]
    u = rng.uniform(-0.02, 0.02, size=net.X.shape)
    g = O.internal_force(net, u)
    h = 1e-6
    for i, k in [(0, 0), (5, 1), (17, 2), (33, 0), (59, 2)]:
        up = u.copy(); up[i, k] += h
        um = u.copy(); um[i, k] -= h
        fd = -(O.energy(net, up) - O.energy(net, um)) / (2 * h)
        assert abs(fd - g[i, k]) < 1e-7 * max(1.0, abs(g[i, k])), (i, k, fd, g[i, k])


def test_converged_stress_symmetric_and_forms_agree(oracle_lib):
    O = oracle_lib
    b = I.config_single()
    net, F = b.nets[0], b.F[0]
    r = O.solve(net, F, tol=1e-8, beta=BETA, dt_safety=S)
    assert r.status == O.CONVERGED
    nrm = np.linalg.norm(r.sigma)
    assert np.linalg.norm(r.sigma - r.sigma.T) < 1e-6 * nrm
    # |sigma - sigma_fib| <= 1/J max|x_i - F c0| sqrt(3 N_f) |g_free|
    d = O.derived(net, BETA, S)
    gb = np.linalg.norm(O.internal_force(net, r.u)[net.fixed == 1])
    gfree = r.rho * max(gb, d["s_floor"])
    x = net.X + r.u
    yc = np.abs(x - F @ np.full(3, 0.5)).max() * math.sqrt(3)
    bound = yc * math.sqrt(3 * (net.n_nodes - net.n_fixed)) * gfree / np.linalg.det(F)
    assert np.linalg.norm(r.sigma - r.sigma_fib) <= bound


# --------------------------------------------------------------------------
# P7: brute-force Newton on small rigid networks (energy minimised with
# torch autograd, independent of the oracle's force routine)
# --------------------------------------------------------------------------
def _newton(net, F):
    import torch
    X = torch.tensor(net.X, dtype=torch.float64)
    fib = torch.tensor(net.fibers, dtype=torch.long)
    EA = torch.tensor(net.EA, dtype=torch.float64)
    L = (X[fib[:, 1]] - X[fib[:, 0]]).norm(dim=1)
    free = torch.tensor(net.fixed == 0)
    Ft = torch.tensor(F, dtype=torch.float64)
    x0 = X @ Ft.T

    def W(xf):
        x = x0.clone()
        x[free] = xf.reshape(-1, 3)
        lam = (x[fib[:, 1]] - x[fib[:, 0]]).norm(dim=1) / L
        return (EA * L * (lam ** 3 - 3 * lam + 2) / 6).sum()

    xf = x0[free].reshape(-1).clone()
    for _ in range(60):
        gr = torch.autograd.functional.jacobian(W, xf)
        if gr.abs().max() < 1e-14:
            break
        H = torch.autograd.functional.hessian(W, xf)
        step = torch.linalg.solve(H, gr)
        t = 1.0
        while W(xf - t * step) > W(xf) + 1e-16 and t > 1e-6:
            t *= 0.5
        xf = xf - t * step
    H = torch.autograd.functional.hessian(W, xf)
    assert torch.linalg.eigvalsh(H).min() > 0  # strict local minimum, unique nearby
    # reactions r_b = dW/dx_b at the solution
    xall = x0.clone(); xall[free] = xf.reshape(-1, 3)
    xall.requires_grad_(True)
    lam = (xall[fib[:, 1]] - xall[fib[:, 0]]).norm(dim=1) / L
    (EA * L * (lam ** 3 - 3 * lam + 2) / 6).sum().backward()
    react = xall.grad.detach().numpy()  # = -g
    x = xall.detach().numpy()
    c0 = F @ np.full(3, 0.5)
    sig = sum(np.outer(react[b], x[b] - c0) for b in np.where(net.fixed == 1)[0]) / np.linalg.det(F)
    return x, sig


@pytest.mark.parametrize("seed", [1, 2])
def test_newton_small_rigid(oracle_lib, seed):
    O = oracle_lib
    rng = np.random.default_rng(seed)
    net = I.complete_network(rng, 9, 4)
    F = np.array([[1.04, 0.01, 0.0], [0.01, 1.02, 0.005], [0.0, 0.005, 1.03]])
    x_ref, sig_ref = _newton(net, F)
    r = O.solve(net, F, tol=1e-12, beta=0.05, dt_safety=S)
    assert r.status == O.CONVERGED
    assert np.abs(net.X + r.u - x_ref).max() < 1e-10
    assert _rel(r.sigma, sig_ref) < 1e-9


# --------------------------------------------------------------------------
# P9: scaling, translation and relabeling
# --------------------------------------------------------------------------
def test_EA_scaling_exact(oracle_lib):
    """EA -> 4 EA: dt halves and c doubles exactly, every iterate is the same
    and the stress is exactly four times larger."""
    O = oracle_lib
    b = I.config_single(150, seed=2)
    net, F = b.nets[0], I.sym_perturbed_F(np.random.default_rng(3), 0.01)
    net4 = I.Network(net.X, net.fibers, 4.0 * net.EA, net.fixed)
    a = O.solve(net, F, tol=1e-8, beta=BETA, dt_safety=S)
    c = O.solve(net4, F, tol=1e-8, beta=BETA, dt_safety=S)
    assert a.iters == c.iters
    assert np.array_equal(a.u, c.u)
    assert np.array_equal(4.0 * a.sigma, c.sigma)
    assert c.dt == a.dt / 2 and c.c == 2 * a.c


def test_translation_and_relabeling(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(4)
    b = I.config_single(150, seed=5)
    net, F = b.nets[0], I.sym_perturbed_F(rng, 0.01)
    a = O.solve(net, F, tol=1e-10, beta=BETA, dt_safety=S)
    t = np.array([0.3, -0.2, 0.1])
    tn = I.Network(net.X + t, net.fibers, net.EA, net.fixed)
    c = O.solve(tn, F, tol=1e-10, beta=BETA, dt_safety=S)
    nrm = np.linalg.norm(a.sigma)
    assert np.linalg.norm(c.sigma - a.sigma) < 1e-7 * nrm
    perm = rng.permutation(net.n_nodes)
    inv = np.argsort(perm)
    fp = rng.permutation(net.n_fibers)
    pn = I.Network(net.X[perm], inv[net.fibers][fp].astype(np.int32), net.EA[fp], net.fixed[perm])
    d = O.solve(pn, F, tol=1e-10, beta=BETA, dt_safety=S)
    assert np.linalg.norm(d.sigma - a.sigma) < 1e-7 * nrm


# --------------------------------------------------------------------------
# P10: no load
# --------------------------------------------------------------------------
def test_identity_no_load(oracle_lib):
    O = oracle_lib
    net = I.config_single().nets[0]
    r = O.solve(net, np.eye(3), tol=1e-8, beta=BETA, dt_safety=S)
    assert r.status == O.CONVERGED and r.iters == 1
    assert np.array_equal(r.u, np.zeros_like(r.u))
    assert np.array_equal(r.sigma, np.zeros((3, 3)))


# --------------------------------------------------------------------------
# Derived constants (readings R2-R4, R6) and failure reporting
# --------------------------------------------------------------------------
def test_derived_constants(oracle_lib):
    O = oracle_lib
    net = _chain()
    d = O.derived(net, 0.02, S)
    mB = 0.5 * (0.25 + 0.35)
    w = math.sqrt(2 / mB * (1.1 * 1.0 / 0.25 + 1.1 * 1.7 / 0.35))
    assert np.allclose(d["m"], [0.125, mB, 0.175])
    assert math.isclose(d["dt"], S * 2 / w, rel_tol=1e-15)
    assert math.isclose(d["c"], 0.02 * w, rel_tol=1e-15)
    assert math.isclose(d["s_floor"], 1e-4 * 1.35 * math.sqrt(6), rel_tol=1e-15)


def test_invalid_and_nonconverged(oracle_lib):
    O = oracle_lib
    net = I.config_single(100, seed=1).nets[0]
    bad = I.Network(net.X, net.fibers, net.EA.copy(), net.fixed)
    bad.EA[3] = 0.0
    with pytest.raises(ValueError):
        O.solve(bad, np.eye(3) * 1.01, beta=BETA, dt_safety=S)
    r = O.solve(net, np.diag([1.02, 1, 1]), tol=1e-8, max_iter=5, beta=BETA, dt_safety=S)
    assert r.status == O.MAX_ITER and r.iters == 5
    # an unstable time step (dt_safety far above the bound) ends NONFINITE
    r = O.solve(net, np.diag([1.02, 1, 1]), tol=1e-8, max_iter=100000, beta=0.0, dt_safety=40.0)
    assert r.status == O.NONFINITE


def test_energy_balance_terms(oracle_lib):
    """Fig. 1's optional energy check.  The trapezoid work of the internal
    forces equals minus the change of the stored energy W = sum EA L
    (lambda^3 - 3 lambda + 2) / 6 (an independent closed form) to the
    scheme's accuracy, and KE - W_int + W_damp stays a small fraction of the
    largest term (a few percent in the first passes, ~1e-3 at convergence)."""
    O = oracle_lib
    b = I.small_batch(2, 100, 300, 0.02, seed=5)
    for i in range(len(b)):
        net, F = b.nets[i], b.F[i]
        E0 = O.energy(net, net.X @ (F - np.eye(3)).T)
        for K, bal_tol in ((50, 0.06), (2000, 3e-3), (None, 3e-3)):
            r = O.solve(net, F, tol=1e-8 if K is None else 1e-30, max_iter=K or 2_000_000, beta=1e-3,
                        dt_safety=0.9)
            dE = O.energy(net, r.u) - E0
            assert abs(r.work_int + dE) <= 2e-3 * abs(dE), (K, r.work_int, dE)
            bal = r.ke - r.work_int + r.work_damp
            assert abs(bal) <= bal_tol * max(r.ke, abs(r.work_int), r.work_damp), (K, bal)
            assert r.work_damp > 0.0


# --------------------------------------------------------------------------
# Fig. 1, "compute next time step" taken literally (reading R16): the step of
# each pass from the current axial tangent stiffness, capped by the constant
# step of R3.
# --------------------------------------------------------------------------
def test_step_rule_closed_form(oracle_lib):
    """One pass from a stretched chain: the step the rule takes equals
    min(dt0, s 2 / w) with w^2 = (2 / m_B)(EA1 l1 / L1^2 + EA2 l2 / L2^2),
    the Gershgorin bound of the middle node at the start state (only the free
    node counts)."""
    O = oracle_lib
    net = _chain()
    F = np.diag([1.8, 1.0, 1.0])
    u0 = np.vstack([F @ x - x for x in net.X])
    u0[1] = [0.12, 0.01, -0.02]  # middle node off the affine position
    r = O.solve(net, F, tol=1e-300, max_iter=1, beta=BETA, dt_safety=S, start=O.START_WARM,
                F_prev=F, u_prev=u0, dt_rule=1)
    x = net.X + u0
    L1, L2 = 0.25, 0.35
    l1 = np.linalg.norm(x[1] - x[0]); l2 = np.linalg.norm(x[2] - x[1])
    mB = 0.5 * (L1 + L2)
    w2 = 2.0 / mB * (net.EA[0] * l1 / L1 ** 2 + net.EA[1] * l2 / L2 ** 2)
    expect = min(r.dt, S * 2.0 / math.sqrt(w2))
    assert expect < r.dt  # the rule is active here
    assert r.dt_min == pytest.approx(expect, rel=1e-14)
    # dt0 of R3 is the same bound with the reference stiffness 1.1 EA / L
    w02 = 2.0 / mB * 1.1 * (net.EA[0] / L1 + net.EA[1] / L2)
    assert r.dt == pytest.approx(S * 2.0 / math.sqrt(w02), rel=1e-14)


def test_step_rule_rescues_a_stretched_start(oracle_lib):
    """The chain stretched four-fold from u = 0: the constant step is too long
    for the stretched fibers' stiffness and the iteration diverges; with the
    per-pass step it converges to the bisection equilibrium."""
    O = oracle_lib
    net = _chain()
    F = np.diag([4.0, 1.0, 1.0])
    a = O.solve(net, F, tol=1e-12, beta=0.05, dt_safety=S, start=O.START_ZERO)
    b = O.solve(net, F, tol=1e-12, beta=0.05, dt_safety=S, start=O.START_ZERO, dt_rule=1)
    assert a.status == O.NONFINITE
    assert b.status == O.CONVERGED and b.dt_min < 0.5 * b.dt
    xB, T, ell, e = _chain_equilibrium(net, F)
    assert np.allclose(net.X[1] + b.u[1], xB, rtol=0, atol=1e-11)


def test_step_rule_keeps_the_constant_step(oracle_lib):
    """Where every fiber's stiffness stays within the 10 % headroom of R3 the
    rule's step is dt0 on every pass and the solve is the constant-step one
    bit for bit."""
    O = oracle_lib
    for batch in (I.config_single(), I.small_batch(3, 80, 300, 0.02, seed=5)):
        for net, F in zip(batch.nets, batch.F):
            a = O.solve(net, F, tol=1e-8, beta=BETA, dt_safety=S)
            b = O.solve(net, F, tol=1e-8, beta=BETA, dt_safety=S, dt_rule=1)
            assert b.dt_min == a.dt == b.dt
            assert a.iters == b.iters and a.status == b.status
            assert np.array_equal(a.u, b.u) and np.array_equal(a.sigma, b.sigma)


def test_evaluate_definitions(oracle_lib):
    """The evaluation of a given state (residual of R6, stress of R7): at the
    state a solve returns it reproduces the solve's own residual and stresses
    bit for bit; at the affine state of the regular lattice the interior is
    in equilibrium and the stress is the closed form."""
    O = oracle_lib
    b = I.small_batch(2, 80, 200, 0.02, seed=6)
    for net, F in zip(b.nets, b.F):
        r = O.solve(net, F, tol=1e-8, beta=BETA, dt_safety=S)
        rho, s, sf = O.evaluate(net, F, r.u)
        assert rho == r.rho and np.array_equal(s, r.sigma) and np.array_equal(sf, r.sigma_fib)
    m = 3
    lat = I.cubic_lattice(m, EA=1.3)
    F = np.array([[1.05, 0.02, 0.0], [0.01, 1.03, 0.0], [0.0, 0.015, 1.04]])
    rho, s, _ = O.evaluate(lat, F, lat.X @ (F - np.eye(3)).T)
    J = np.linalg.det(F)
    sig = sum((m + 1) ** 2 / J * 1.3 * (np.linalg.norm(F[:, k]) ** 2 - 1) / (2 * np.linalg.norm(F[:, k]))
              * np.outer(F[:, k], F[:, k]) for k in range(3))
    assert rho < 1e-13
    assert _rel(s, sig) < 1e-12
