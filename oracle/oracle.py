"""ctypes front end of the plain-C FP64 dynamic-relaxation oracle.

TEST INFRASTRUCTURE ONLY: the product path never imports this module.

The arithmetic lives in ``dr_oracle.c`` (Fig. 1 of the paper, step by step);
this file only builds that library with gcc, marshals numpy arrays and runs
independent problems on a thread pool (ctypes drops the GIL during the call).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass
from typing import Optional

import numpy as np

CONVERGED, MAX_ITER, NONFINITE = 0, 1, 2
START_AFFINE, START_ZERO, START_WARM = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dr_oracle.c")
_LIB = os.path.join(_HERE, "libdr_oracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_bp = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile dr_oracle.c with gcc (no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-std=c99", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = C.CDLL(_LIB)
        lib.oracle_solve.restype = C.c_int
        lib.oracle_solve.argtypes = [
            C.c_int, _dp, C.c_int, _ip, _dp, _bp, _dp,
            C.c_int, C.c_void_p, C.c_void_p,
            C.c_double, C.c_long, C.c_double, C.c_double,
            _dp, _dp, _dp, C.POINTER(C.c_long),
            C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
            C.c_void_p, C.c_long, _dp, C.c_int]
        lib.oracle_internal_force.restype = None
        lib.oracle_internal_force.argtypes = [C.c_int, _dp, _dp, C.c_int, _ip, _dp, _dp, _dp]
        lib.oracle_evaluate.restype = C.c_int
        lib.oracle_evaluate.argtypes = [C.c_int, _dp, _dp, C.c_int, _ip, _dp, _bp, _dp,
                                        C.POINTER(C.c_double), _dp, _dp]
        lib.oracle_energy.restype = C.c_double
        lib.oracle_energy.argtypes = [C.c_int, _dp, _dp, C.c_int, _ip, _dp, _dp]
        lib.oracle_derived.restype = C.c_int
        lib.oracle_derived.argtypes = [C.c_int, _dp, C.c_int, _ip, _dp, _bp, C.c_double, C.c_double,
                                       _dp, _dp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double)]
        _lib = lib
    return _lib


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


@dataclass
class OracleResult:
    status: int
    u: np.ndarray          # (N, 3)
    sigma: np.ndarray      # (3, 3) boundary (reaction) form
    sigma_fib: np.ndarray  # (3, 3) fiber form
    iters: int
    rho: float
    ke: float
    dt: float
    c: float
    rho_trace: Optional[np.ndarray] = None
    work_int: float = 0.0   # work of the internal forces over the solve (trapezoid per pass)
    work_damp: float = 0.0  # work dissipated by the damping force
    dt_min: float = 0.0     # smallest step used (the constant step unless dt_rule = 1)


def derived(net, beta: float, dt_safety: float):
    """Fiber lengths, lumped masses, dt, c and the residual floor."""
    lib = _load()
    N, M = net.n_nodes, net.n_fibers
    L = np.zeros(max(M, 1)); m = np.zeros(N)
    dt, c, fl = C.c_double(), C.c_double(), C.c_double()
    rc = lib.oracle_derived(N, _c(net.X, np.float64).ravel(), M, _c(net.fibers, np.int32).ravel(),
                            _c(net.EA, np.float64), _c(net.fixed, np.uint8), beta, dt_safety,
                            L, m, C.byref(dt), C.byref(c), C.byref(fl))
    if rc != 0:
        raise ValueError("oracle_derived: invalid network (%d)" % rc)
    return dict(L=L[:M], m=m, dt=dt.value, c=c.value, s_floor=fl.value)


def internal_force(net, u: np.ndarray) -> np.ndarray:
    lib = _load()
    N, M = net.n_nodes, net.n_fibers
    X = _c(net.X, np.float64).ravel()
    fib = _c(net.fibers, np.int32).ravel()
    L = np.linalg.norm(net.X[net.fibers[:, 1]] - net.X[net.fibers[:, 0]], axis=1)
    g = np.zeros(3 * N)
    lib.oracle_internal_force(N, X, _c(u, np.float64).ravel(), M, fib, _c(net.EA, np.float64),
                              _c(L, np.float64), g)
    return g.reshape(N, 3)


def energy(net, u: np.ndarray) -> float:
    lib = _load()
    N, M = net.n_nodes, net.n_fibers
    L = np.linalg.norm(net.X[net.fibers[:, 1]] - net.X[net.fibers[:, 0]], axis=1)
    return lib.oracle_energy(N, _c(net.X, np.float64).ravel(), _c(u, np.float64).ravel(), M,
                             _c(net.fibers, np.int32).ravel(), _c(net.EA, np.float64), _c(L, np.float64))


def evaluate(net, F, u: np.ndarray):
    """Residual rho (reading R6) and both stress forms (R7) of the state u
    (N x 3 displacements, prescribed nodes as given) under F, without
    iterating: whether a state returned by another solver is an equilibrium,
    and what its stress is, by this file's definitions."""
    lib = _load()
    N, M = net.n_nodes, net.n_fibers
    rho = C.c_double()
    sig = np.zeros(9); sigf = np.zeros(9)
    rc = lib.oracle_evaluate(N, _c(net.X, np.float64).ravel(), _c(u, np.float64).ravel(), M,
                             _c(net.fibers, np.int32).ravel(), _c(net.EA, np.float64),
                             _c(net.fixed, np.uint8), _c(F, np.float64).ravel(), C.byref(rho), sig, sigf)
    if rc != 0:
        raise ValueError("oracle_evaluate: invalid input (%d)" % rc)
    return rho.value, sig.reshape(3, 3), sigf.reshape(3, 3)


def solve(net, F, *, tol=1e-8, max_iter=2_000_000, beta, dt_safety,
          start=START_AFFINE, F_prev=None, u_prev=None, trace_len: int = 0,
          dt_rule: int = 0) -> OracleResult:
    """One DR solve of ``net`` under deformation gradient ``F`` (3x3).
    dt_rule 0: constant step (reading R3); 1: per-pass step (reading R16)."""
    lib = _load()
    N, M = net.n_nodes, net.n_fibers
    X = _c(net.X, np.float64).ravel()
    fib = _c(net.fibers, np.int32).ravel()
    EA = _c(net.EA, np.float64)
    fixed = _c(net.fixed, np.uint8)
    Fa = _c(F, np.float64).ravel()
    keep = []
    Fp = up = None
    if start == START_WARM:
        Fpa = _c(F_prev, np.float64).ravel(); upa = _c(u_prev, np.float64).ravel()
        keep += [Fpa, upa]
        Fp, up = Fpa.ctypes.data, upa.ctypes.data
    u = np.zeros(3 * N); sig = np.zeros(9); sigf = np.zeros(9)
    it = C.c_long(); rho = C.c_double(); ke = C.c_double(); dt = C.c_double(); c = C.c_double()
    tr = np.zeros(max(trace_len, 1)) if trace_len > 0 else None
    work = np.zeros(3)
    rc = lib.oracle_solve(N, X, M, fib, EA, fixed, Fa, int(start), Fp, up,
                          float(tol), int(max_iter), float(beta), float(dt_safety),
                          u, sig, sigf, C.byref(it), C.byref(rho), C.byref(ke), C.byref(dt), C.byref(c),
                          tr.ctypes.data if tr is not None else None, int(trace_len), work,
                          int(dt_rule))
    if rc < 0:
        raise ValueError("oracle_solve: invalid input (%d)" % rc)
    return OracleResult(rc, u.reshape(N, 3), sig.reshape(3, 3), sigf.reshape(3, 3), it.value,
                        rho.value, ke.value, dt.value, c.value,
                        tr[:min(it.value, trace_len)] if tr is not None else None,
                        float(work[0]), float(work[1]), float(work[2]))


def solve_batch(batch, *, threads: Optional[int] = None, **kw):
    """Solve every network of a Batch, one problem per thread."""
    _load()
    threads = threads or os.cpu_count() or 1
    jobs = list(range(len(batch)))
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda i: solve(batch.nets[i], batch.F[i], **kw), jobs))
