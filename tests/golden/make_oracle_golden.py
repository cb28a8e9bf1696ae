#!/usr/bin/env python3
"""Writes the oracle's results that the GPU parity tests compare against.

Only the CPU oracle (oracle/) and the seeded input generators are used; no
value here comes from the HIP path.  The files it writes:

  uniform256_sample.json   the 256-network workload (N ~ U{1000..5000},
      F = I + sym U(+-0.01), damping 1e-4, dt_safety 0.9): a stratified
      sample of 16 networks (the slowest to converge, the largest, the
      smallest and three from the middle of the size range) solved at tol
      1e-8 and 1e-10, each also from four starts perturbed by 1e-15 (normal,
      on the free nodes), which measures how far the iteration's own
      rounding moves the equilibrium it reaches;
  uniform256_all.json      every network of that workload at tol 1e-8
      (stress, passes, residual, status);
  uneven1024_sample.json   the 1024-network workload (N log-uniform in
      [2000, 33000], F = I + sym U(+-0.02), damping 1e-4): two networks of
      each default size class (register/LDS up to 6720 nodes, global above)
      at tol 1e-8, with three perturbed starts each;
  uneven1024_steprule.json   the four networks of that workload (indices
      248, 278, 325, 425) whose constant-step solves diverge (a fiber
      stretched beyond the step's headroom), solved with the per-pass step
      (dt_rule 1) at tol 1e-8, with two perturbed starts each.

Usage: python tests/golden/make_oracle_golden.py [uniform_sample|uniform_all|uneven_sample|uneven_steprule ...]
(all three by default).  Runs one problem per thread on all host threads
but one; the full set takes about an hour of CPU time per thread.
"""
from __future__ import annotations

import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2305_07030_amd import inputs as I  # noqa: E402

BETA = 1e-4
DT_SAFETY = 0.9
N_PERTURBED_UNIFORM = 4
N_PERTURBED_UNEVEN = 3
PERTURBATION = 1e-15
MAX_ITER = 4_000_000

# Networks of the 256-network workload whose solves take the most passes
# (the ones that set the batch's wall time), by index.
UNIFORM_SLOW = [103, 24, 225, 70, 99]


def perturbed_start(net, F, k):
    """Affine start plus a 1e-15 normal perturbation of the free nodes."""
    u0 = net.X @ (F - np.eye(3)).T
    noise = np.random.default_rng(1000 + k).normal(size=u0.shape) * PERTURBATION
    return u0 + noise * (net.fixed == 0)[:, None]


def solve_one(net, F, tol, k, dt_rule=0):
    """k < 0: the plain affine start; k >= 0: perturbed start number k."""
    kw = dict(tol=tol, max_iter=MAX_ITER, beta=BETA, dt_safety=DT_SAFETY, dt_rule=dt_rule)
    if k >= 0:
        kw.update(start=O.START_WARM, F_prev=F, u_prev=perturbed_start(net, F, k))
    t = time.perf_counter()
    r = O.solve(net, F, **kw)
    return dict(sigma=r.sigma.ravel().tolist(), sigma_fib=r.sigma_fib.ravel().tolist(),
                iters=int(r.iters), rho=float(r.rho), status=int(r.status), dt_min=float(r.dt_min),
                seconds=round(time.perf_counter() - t, 2))


def run_jobs(jobs, threads, label, dt_rule=0):
    """jobs: list of (key, net, F, tol, k, cost).  Longest first."""
    jobs = sorted(jobs, key=lambda j: -j[5])
    out = {}
    t0 = time.perf_counter()
    done = [0]

    def work(j):
        key, net, F, tol, k, _ = j
        r = solve_one(net, F, tol, k, dt_rule)
        done[0] += 1
        print(f"[{label}] {done[0]}/{len(jobs)} {key} tol {tol:g} start {k}: {r['iters']} passes, "
              f"status {r['status']}, {r['seconds']}s (t={time.perf_counter() - t0:.0f}s)", flush=True)
        return j, r

    with ThreadPoolExecutor(max_workers=threads) as ex:
        for j, r in ex.map(work, jobs):
            out[(j[0], j[3], j[4])] = r
    return out


def uniform_sample_ids(sizes):
    """{index: why} for the stratified sample of the 256-network workload."""
    order = np.argsort(sizes, kind="stable")
    why = {}
    for i in UNIFORM_SLOW:
        why.setdefault(i, "slowest")
    for i in order[::-1][:5]:
        why.setdefault(int(i), "largest")
    for i in order[:3]:
        why.setdefault(int(i), "smallest")
    # the rest from the middle of the size range
    for i in order[len(order) // 2 - 8:len(order) // 2 + 8]:
        if len(why) >= 16:
            break
        why.setdefault(int(i), "middle")
    return why


def uniform_sample(threads):
    full = I.config_uniform_batch(256)
    sizes = np.array([n.n_nodes for n in full.nets])
    why = uniform_sample_ids(sizes)
    ids = list(why)
    jobs = []
    for i in ids:
        net, F = full.nets[i], full.F[i]
        cost = net.n_fibers * (3.0 if i in UNIFORM_SLOW else 1.0)
        for tol in (1e-8, 1e-10):
            for k in [-1] + list(range(N_PERTURBED_UNIFORM)):
                jobs.append((i, net, F, tol, k, cost * (1.5 if tol < 1e-9 else 1.0)))
    res = run_jobs(jobs, threads, "uniform-sample")
    nets = []
    for i in ids:
        e = dict(index=i, n_nodes=int(sizes[i]), n_fibers=full.nets[i].n_fibers, why=why[i])
        for tol in (1e-8, 1e-10):
            e[f"tol_{tol:g}"] = dict(plain=res[(i, tol, -1)],
                                     perturbed=[res[(i, tol, k)] for k in range(N_PERTURBED_UNIFORM)])
        nets.append(e)
    return dict(workload="256 kNN(k=3) networks, N ~ U{1000..5000}, F = I + sym U(+-0.01), "
                         "SeedSequence(2)", damping=BETA, dt_safety=DT_SAFETY, max_iter=MAX_ITER,
                perturbation=PERTURBATION, networks=nets)


def uniform_all(threads):
    full = I.config_uniform_batch(256)
    jobs = [(i, full.nets[i], full.F[i], 1e-8, -1, full.nets[i].n_fibers) for i in range(len(full))]
    res = run_jobs(jobs, threads, "uniform-all")
    return dict(workload="256 kNN(k=3) networks, N ~ U{1000..5000}, F = I + sym U(+-0.01), "
                         "SeedSequence(2)", damping=BETA, dt_safety=DT_SAFETY, tol=1e-8,
                max_iter=MAX_ITER,
                networks=[dict(index=i, n_nodes=full.nets[i].n_nodes, **res[(i, 1e-8, -1)])
                          for i in range(len(full))])


def uneven_sizes(P=1024):
    """Node counts of the 1024-network workload (the first draw of each
    network's generator)."""
    seqs = np.random.SeedSequence(3).spawn(P)
    out = []
    for s in seqs:
        rng = np.random.default_rng(s)
        out.append(int(round(np.exp(rng.uniform(np.log(2000), np.log(33000))))))
    return np.array(out)


def uneven_sample(threads):
    sizes = uneven_sizes()
    targets = [3000, 6000, 12000, 24000]
    ids = []
    for t in targets:
        i = int(np.argmin(np.abs(sizes - t)))
        ids.append(i)
    sub = I.config_uneven_batch(1024, idx=ids)
    jobs = []
    for k_net, i in enumerate(ids):
        net, F = sub.nets[k_net], sub.F[k_net]
        for k in [-1] + list(range(N_PERTURBED_UNEVEN)):
            jobs.append((i, net, F, 1e-8, k, net.n_fibers))
    res = run_jobs(jobs, threads, "uneven-sample")
    nets = []
    for k_net, i in enumerate(ids):
        nets.append(dict(index=i, n_nodes=sub.nets[k_net].n_nodes, n_fibers=sub.nets[k_net].n_fibers,
                         **{"tol_1e-08": dict(plain=res[(i, 1e-8, -1)],
                                       perturbed=[res[(i, 1e-8, k)] for k in range(N_PERTURBED_UNEVEN)])}))
    return dict(workload="1024 kNN(k=3) networks, N = round(exp U(ln 2000, ln 33000)), "
                         "F = I + sym U(+-0.02), SeedSequence(3)", damping=BETA, dt_safety=DT_SAFETY,
                max_iter=MAX_ITER, perturbation=PERTURBATION, networks=nets)


UNEVEN_DIVERGING = [248, 278, 325, 425]


def uneven_steprule(threads):
    ids = UNEVEN_DIVERGING
    sub = I.config_uneven_batch(1024, idx=ids)
    jobs = []
    for k_net, i in enumerate(ids):
        net, F = sub.nets[k_net], sub.F[k_net]
        for k in [-1, 0, 1]:
            jobs.append((i, net, F, 1e-8, k, net.n_fibers))
    res = run_jobs(jobs, threads, "uneven-steprule", dt_rule=1)
    nets = []
    for k_net, i in enumerate(ids):
        nets.append(dict(index=i, n_nodes=sub.nets[k_net].n_nodes, n_fibers=sub.nets[k_net].n_fibers,
                         **{"tol_1e-08": dict(plain=res[(i, 1e-8, -1)],
                                              perturbed=[res[(i, 1e-8, k)] for k in range(2)])}))
    return dict(workload="1024 kNN(k=3) networks, N = round(exp U(ln 2000, ln 33000)), "
                         "F = I + sym U(+-0.02), SeedSequence(3); per-pass step (dt_rule 1)",
                damping=BETA, dt_safety=DT_SAFETY, max_iter=MAX_ITER, perturbation=PERTURBATION,
                dt_rule=1, networks=nets)


def main():
    what = sys.argv[1:] or ["uniform_sample", "uniform_all", "uneven_sample"]
    threads = max(1, int(os.environ.get("GOLDEN_THREADS", (os.cpu_count() or 2) - 1)))
    O.build(force=False)
    makers = dict(uniform_sample=(uniform_sample, "uniform256_sample.json"),
                  uniform_all=(uniform_all, "uniform256_all.json"),
                  uneven_sample=(uneven_sample, "uneven1024_sample.json"),
                  uneven_steprule=(uneven_steprule, "uneven1024_steprule.json"))
    for w in what:
        fn, name = makers[w]
        t = time.perf_counter()
        data = fn(threads)
        data["generated_by"] = "tests/golden/make_oracle_golden.py " + w
        data["oracle"] = "oracle/dr_oracle.c (gcc -O2 -ffp-contract=off)"
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(data, f, indent=1)
        print(f"wrote {name} in {time.perf_counter() - t:.0f}s", flush=True)


if __name__ == "__main__":
    main()
