"""Macroscale tangent of the microscale stress by perturbation solves.

In the FE2 setting of section I the macroscale solver needs, besides the
stress, its derivative with respect to the deformation gradient at each
material point.  The sub-problem gives it by finite differences: for each of
the six symmetric directions E_kl = (e_k e_l^T + e_l e_k^T) / 2, two
warm-started solves at F + h E_kl and F - h E_kl give

    D[:, :, k, l] = D[:, :, l, k] = (sigma(F + h E_kl) - sigma(F - h E_kl)) / (2 h),

the derivative of sigma along symmetric perturbations of F.  Every solve
starts from the displacements the previous one left on the device
(DR_START_WARM), the first from the converged state at F.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from . import dr

DIRECTIONS: List[Tuple[int, int]] = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


def sym_dir(k: int, l: int) -> np.ndarray:
    E = np.zeros((3, 3))
    E[k, l] += 0.5
    E[l, k] += 0.5
    return E


def tangent(b: "dr.DRBatch", F: np.ndarray, h: float = 1e-3) -> dict:
    """Tangent of every problem of the batch at F [P, 3, 3].  Returns sigma
    at F [P, 3, 3], the tangent [P, 3, 3, 3, 3] and the passes spent."""
    F = np.asarray(F, np.float64).reshape(-1, 3, 3)
    P = F.shape[0]
    b.solve(F=F, start=dr.DR_START_AFFINE)
    r0 = b.results()
    passes = r0["iters"].astype(np.int64).copy()
    results = [r0["result"].copy()]
    D = np.zeros((P, 3, 3, 3, 3))
    for k, l in DIRECTIONS:
        E = sym_dir(k, l)
        sig = []
        for sgn in (1.0, -1.0):
            b.solve(F=F + sgn * h * E, start=dr.DR_START_WARM)
            r = b.results()
            passes += r["iters"]
            results.append(r["result"].copy())
            sig.append(r["sigma"])
        d = (sig[0] - sig[1]) / (2.0 * h)
        D[:, :, :, k, l] = d
        D[:, :, :, l, k] = d
    return dict(sigma=r0["sigma"], D=D, passes=passes, results=np.stack(results))
