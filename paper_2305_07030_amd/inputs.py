"""Seeded synthetic fiber-network workloads.

This module only *draws* inputs: node coordinates, fiber connectivity, fiber
stiffness EA, the prescribed-node mask and the macroscale deformation gradient
F.  It holds none of the dynamic-relaxation arithmetic, so both the HIP path
and the CPU oracle can be fed from it without sharing any solver code.

The paper solves athermal collagen fiber networks (section II); its networks
are not published, so random networks of the same kind stand in for them:

* nodes uniform in the unit cube, each joined to its k = 3 nearest other
  nodes (Euclidean, non-periodic), undirected union, duplicates removed,
  fibers stored with a < b and sorted;
* EA lognormal with E[EA] = 1 and log-standard-deviation 0.2, drawn in sorted
  fiber order after the coordinates;
* a node is prescribed ("fixed") when it lies within ``band`` = 0.02 of any
  face of the cube (inclusive);
* F = I + a symmetric perturbation whose six upper-triangle entries are drawn
  i.i.d. U(-a, a) in the order 11, 12, 13, 22, 23, 33 and mirrored.

Batches are drawn per network from ``SeedSequence(base).spawn(P)[r]`` in the
order: node count, coordinates, EA, F entries.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
from scipy.spatial import cKDTree

EA_LOG_SIGMA = 0.2
EA_LOG_MU = -0.5 * EA_LOG_SIGMA ** 2  # E[EA] = exp(mu + s^2/2) = 1
BAND = 0.02


@dataclass
class Network:
    """One sub-problem: a pin-jointed fiber network in the unit cube."""
    X: np.ndarray          # (N, 3) float64 reference coordinates
    fibers: np.ndarray     # (M, 2) int32 node ids, a < b
    EA: np.ndarray         # (M,) float64 axial stiffness
    fixed: np.ndarray      # (N,) uint8, 1 = prescribed node

    @property
    def n_nodes(self) -> int:
        return int(self.X.shape[0])

    @property
    def n_fibers(self) -> int:
        return int(self.fibers.shape[0])

    @property
    def n_fixed(self) -> int:
        return int(self.fixed.sum())


@dataclass
class Batch:
    """Many independent networks, each with its own deformation gradient."""
    nets: List[Network]
    F: np.ndarray                      # (P, 3, 3) float64, F_ij = dx_i / dX_j
    name: str = ""
    meta: dict = field(default_factory=dict)

    def __len__(self) -> int:
        return len(self.nets)

    def packed(self):
        """Concatenate the networks into flat arrays (CSR-style offsets).

        Returns a dict with node_offsets[P+1], fiber_offsets[P+1] (int64),
        X[sum N, 3], fiber_nodes[sum M, 2] (problem-local ids, int32),
        EA[sum M], fixed[sum N] (uint8).
        """
        P = len(self.nets)
        no = np.zeros(P + 1, np.int64)
        fo = np.zeros(P + 1, np.int64)
        for i, n in enumerate(self.nets):
            no[i + 1] = no[i] + n.n_nodes
            fo[i + 1] = fo[i] + n.n_fibers
        return dict(
            node_offsets=no,
            fiber_offsets=fo,
            X=np.ascontiguousarray(np.concatenate([n.X for n in self.nets]), dtype=np.float64),
            fiber_nodes=np.ascontiguousarray(np.concatenate([n.fibers for n in self.nets]), dtype=np.int32),
            EA=np.ascontiguousarray(np.concatenate([n.EA for n in self.nets]), dtype=np.float64),
            fixed=np.ascontiguousarray(np.concatenate([n.fixed for n in self.nets]), dtype=np.uint8),
        )

    def subset(self, idx: Sequence[int]) -> "Batch":
        idx = list(idx)
        return Batch([self.nets[i] for i in idx], self.F[idx].copy(), self.name + "[sub]", dict(self.meta))

    @property
    def total_fibers(self) -> int:
        return int(sum(n.n_fibers for n in self.nets))

    @property
    def total_nodes(self) -> int:
        return int(sum(n.n_nodes for n in self.nets))


# --------------------------------------------------------------------------
# network construction
# --------------------------------------------------------------------------

def knn_fibers(X: np.ndarray, k: int = 3) -> np.ndarray:
    """Undirected union of each node's k nearest *other* nodes.

    Returns (M, 2) int32 with a < b, rows sorted lexicographically."""
    N = X.shape[0]
    if N < 2:
        return np.zeros((0, 2), np.int32)
    kk = min(k + 1, N)
    _, nb = cKDTree(X).query(X, k=kk)
    nb = np.asarray(nb).reshape(N, kk)
    rows = []
    for j in range(1, kk):
        a = np.arange(N)
        b = nb[:, j]
        rows.append(np.stack([np.minimum(a, b), np.maximum(a, b)], 1))
    e = np.concatenate(rows)
    e = e[e[:, 0] != e[:, 1]]
    e = np.unique(e, axis=0)
    return e.astype(np.int32)


def band_fixed(X: np.ndarray, band: float = BAND) -> np.ndarray:
    """1 where a node lies within ``band`` of any face of the unit cube."""
    d = np.minimum(X, 1.0 - X).min(axis=1)
    return (d <= band).astype(np.uint8)


def draw_network(rng: np.random.Generator, n_nodes: int, k: int = 3, band: float = BAND) -> Network:
    X = rng.random((n_nodes, 3))
    fib = knn_fibers(X, k)
    EA = rng.lognormal(EA_LOG_MU, EA_LOG_SIGMA, size=fib.shape[0])
    return Network(X, fib, EA.astype(np.float64), band_fixed(X, band))


def sym_perturbed_F(rng: np.random.Generator, amp: float) -> np.ndarray:
    e = rng.uniform(-amp, amp, size=6)
    F = np.eye(3)
    F[0, 0] += e[0]; F[0, 1] += e[1]; F[0, 2] += e[2]
    F[1, 1] += e[3]; F[1, 2] += e[4]; F[2, 2] += e[5]
    F[1, 0] = F[0, 1]; F[2, 0] = F[0, 2]; F[2, 1] = F[1, 2]
    return F


def _loguniform_int(rng: np.random.Generator, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def config_single(n_nodes: int = 500, seed: int = 0) -> Batch:
    """One 500-node network, F = diag(1.01, 1, 1), seed 0."""
    rng = np.random.default_rng(seed)
    net = draw_network(rng, n_nodes)
    F = np.diag([1.01, 1.0, 1.0])[None].copy()
    return Batch([net], F, f"single-N{n_nodes}-seed{seed}", dict(tol=1e-8))


def _spawned_batch(base: int, P: int, size_fn, amp: float, name: str, idx=None) -> Batch:
    seqs = np.random.SeedSequence(base).spawn(P)
    idx = range(P) if idx is None else idx
    nets, Fs = [], []
    for r in idx:
        rng = np.random.default_rng(seqs[r])
        N = size_fn(rng)
        nets.append(draw_network(rng, N))
        Fs.append(sym_perturbed_F(rng, amp))
    return Batch(nets, np.stack(Fs), name)


def config_uniform_batch(P: int = 256, idx=None) -> Batch:
    """P networks, N ~ U{1000..5000}, F = I + sym U(+-0.01); seed base 2."""
    b = _spawned_batch(2, P, lambda r: int(r.integers(1000, 5001)), 0.01,
                       f"uniform-1000-5000-P{P}", idx)
    b.meta["tol"] = 1e-8
    return b


def config_uneven_batch(P: int = 1024, idx=None) -> Batch:
    """P networks, N log-uniform in [2000, 33000], F = I + sym U(+-0.02); seed base 3."""
    b = _spawned_batch(3, P, lambda r: _loguniform_int(r, 2000, 33000), 0.02,
                       f"loguniform-2000-33000-P{P}", idx)
    b.meta["tol"] = 1e-8
    return b


def config_pool(P: int = 4096, idx=None) -> Batch:
    """Serving pool: N log-uniform in [1000, 33000]; seed base 5."""
    b = _spawned_batch(5, P, lambda r: _loguniform_int(r, 1000, 33000), 0.02,
                       f"pool-loguniform-1000-33000-P{P}", idx)
    return b


def small_batch(P: int, n_lo: int, n_hi: int, amp: float, seed: int) -> Batch:
    """A batch of small kNN networks for quick parity tests."""
    return _spawned_batch(seed, P, lambda r: int(r.integers(n_lo, n_hi + 1)), amp,
                          f"small-{n_lo}-{n_hi}-P{P}-s{seed}")


# --------------------------------------------------------------------------
# structured networks used by the closed-form checks
# --------------------------------------------------------------------------

def cubic_lattice(m: int, EA: float = 1.0) -> Network:
    """(m+1)^3 nodes on a regular grid of spacing 1/m, fibers along the axes.

    Only face nodes are prescribed when 1/m > BAND."""
    g = np.arange(m + 1) / m
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    idx = np.arange((m + 1) ** 3).reshape(m + 1, m + 1, m + 1)
    fib = []
    for ax in range(3):
        a = np.take(idx, range(m), axis=ax).ravel()
        b = np.take(idx, range(1, m + 1), axis=ax).ravel()
        fib.append(np.stack([a, b], 1))
    fib = np.concatenate(fib)
    fib = np.stack([fib.min(1), fib.max(1)], 1)
    fib = np.unique(fib, axis=0).astype(np.int32)
    return Network(X, fib, np.full(fib.shape[0], float(EA)), band_fixed(X))


def complete_network(rng: np.random.Generator, n_nodes: int, n_fixed: int,
                     EA_spread: float = 0.2) -> Network:
    """Complete graph on n_nodes random points; the first n_fixed are prescribed."""
    X = rng.random((n_nodes, 3))
    a, b = np.triu_indices(n_nodes, 1)
    fib = np.stack([a, b], 1).astype(np.int32)
    EA = rng.lognormal(EA_LOG_MU, EA_spread, size=fib.shape[0])
    fixed = np.zeros(n_nodes, np.uint8)
    fixed[:n_fixed] = 1
    return Network(X, fib, EA, fixed)


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])
