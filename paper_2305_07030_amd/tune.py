"""Launch-shape autotuner for batches of uneven size.

The paper runs every sub-problem with one fixed team size (section IV); on
gfx950 the best shape depends on the node count: how many nodes each lane
holds, whether the nodal state fits in LDS, and how many workgroups share a
compute unit.  The tuner splits a batch's node-count range into buckets,
times every valid plan (block, chunk, placement) on a sample of each bucket's
own problems at a fixed pass count, and hands the fastest plan per bucket to
dr_set_class_plans before the batch's first solve.

What is timed is one launch over the sample, all problems at the same pass
count, so a plan's score carries both its per-pass latency and how many of
its workgroups fit on a compute unit at once.  Only the launch shape changes
between candidates: every plan computes the same iteration.

Results are cached in memory and, if a path is given, in a JSON file keyed by
device architecture, compute-unit count, precision and bucket bounds.
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import dataclass
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import dr

# Upper bucket bounds (inclusive).  6720 is the largest FP64 problem whose
# nodal state fits the 160 KiB LDS of one compute unit with 1024 lanes, so it
# separates the LDS-resident and global placements.
DEFAULT_EDGES = (256, 512, 1024, 2048, 4096, 6720, 8192, 16384, 32768)
BLOCKS = (256, 512, 1024)
CHUNKS = (1, 2, 4)


@dataclass(frozen=True)
class Plan:
    block: int
    chunk: int
    placement: int

    def as_dict(self, n_hi: int) -> dict:
        return dict(n_hi=int(n_hi), block=self.block, chunk=self.chunk, placement=self.placement)


def buckets(sizes: Sequence[int], edges: Sequence[int] = DEFAULT_EDGES) -> List[Tuple[int, int, np.ndarray]]:
    """Non-empty buckets (lo, hi, member indices) covering all sizes; bucket k
    is (edges[k-1], edges[k]], the last one ends at the largest size."""
    sizes = np.asarray(sizes)
    bounds = [e for e in sorted(set(int(e) for e in edges)) if e < sizes.max()] + [int(sizes.max())]
    out, lo = [], 1
    for hi in bounds:
        idx = np.nonzero((sizes >= lo) & (sizes <= hi))[0]
        if len(idx):
            out.append((lo, hi, idx))
        lo = hi + 1
    return out


def candidates(n_max: int) -> List[Plan]:
    """Plans worth timing for a bucket whose largest problem has n_max nodes
    (the library rejects the ones whose LDS state does not fit)."""
    out = []
    for blk in BLOCKS:
        if blk > 256 and blk > 2 * n_max:
            continue  # more lanes than twice the nodes: idle lanes only
        for ch in CHUNKS:
            out.append(Plan(blk, ch, dr.DR_PLACE_LDS))
        out.append(Plan(blk, 4, dr.DR_PLACE_GLOBAL))
    return out


def sample(sizes: np.ndarray, idx: np.ndarray, k: int) -> np.ndarray:
    """Up to k members of a bucket spread over its size range, always
    including its largest problem."""
    if len(idx) <= k:
        return idx
    order = idx[np.argsort(sizes[idx], kind="stable")]
    pick = np.unique(np.linspace(0, len(order) - 1, k).round().astype(int))
    return order[pick]


def device_key(precision: int) -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return f"{getattr(p, 'gcnArchName', p.name)}|cu{p.multi_processor_count}|prec{precision}"


def time_plan(sub, plan: Plan, *, passes: int, precision: int, reps: int,
              clock: Callable[[], float] = time.perf_counter) -> Optional[float]:
    """Median wall time of one fixed-pass launch over the sub-batch with this
    plan, or None when the library rejects the plan for it or a problem of the
    sample does not complete the passes."""
    n_hi = max(n.n_nodes for n in sub.nets)
    b = dr.DRBatch(sub, tol=1e-300, max_iter=passes, precision=precision)
    try:
        try:
            b.set_class_plans([plan.as_dict(n_hi)])
        except dr.DrError as e:
            if e.status == dr.DR_E_INVALID:
                return None
            raise
        b.solve()
        b.sync()  # warm-up
        # a plan must run the sample's passes to the end (no early stop)
        if not (b.results()["result"] == dr.DR_MAX_ITER).all():
            return None
        ts = []
        for _ in range(reps):
            t0 = clock()
            b.solve()
            b.sync()
            ts.append(clock() - t0)
        return float(np.median(ts))
    finally:
        b.close()


class Tuner:
    def __init__(self, *, edges: Sequence[int] = DEFAULT_EDGES, passes: int = 1000,
                 sample_size: int = 64, reps: int = 3, cache_path: Optional[str] = None,
                 timer: Callable = time_plan, key: Optional[Callable[[int], str]] = None,
                 log: Callable[[str], None] = lambda s: None):
        self.edges = tuple(edges)
        self.passes = int(passes)
        self.sample_size = int(sample_size)
        self.reps = int(reps)
        self.cache_path = cache_path
        self.timer = timer
        self.key = key or device_key
        self.log = log
        self.cache: Dict[str, dict] = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    def _save(self):
        if self.cache_path:
            os.makedirs(os.path.dirname(os.path.abspath(self.cache_path)), exist_ok=True)
            tmp = self.cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)
            os.replace(tmp, self.cache_path)

    def tune(self, batch, precision: int = dr.DR_FP64) -> List[dict]:
        """Class plans (ascending n_hi) for dr_set_class_plans; each entry also
        carries the bucket's measured times under 'times'."""
        sizes = np.array([n.n_nodes for n in batch.nets])
        dkey = self.key(precision)
        plans = []
        for lo, hi, idx in buckets(sizes, self.edges):
            ckey = f"{dkey}|{lo}-{hi}|K{self.passes}"
            if ckey not in self.cache:
                sub = batch.subset(sample(sizes, idx, self.sample_size))
                n_max = int(sizes[idx].max())
                times = {}
                for pl in candidates(n_max):
                    t = self.timer(sub, pl, passes=self.passes, precision=precision, reps=self.reps)
                    if t is not None:
                        times[f"{pl.block}/{pl.chunk}/{pl.placement}"] = t
                        self.log(f"bucket ({lo},{hi}] n={len(sub)} plan {pl}: {t * 1e3:.3f} ms")
                if not times:
                    raise dr.DrError(dr.DR_E_INVALID, f"no valid plan for bucket ({lo},{hi}]")
                best = min(times, key=times.get)
                self.cache[ckey] = dict(best=best, times=times, sample=len(sub))
                self._save()
            ent = self.cache[ckey]
            blk, ch, place = (int(x) for x in ent["best"].split("/"))
            plans.append(dict(n_hi=int(hi), block=blk, chunk=ch, placement=place,
                              times=dict(ent["times"])))
        return plans


def apply(b: "dr.DRBatch", plans: List[dict]):
    """Install tuned class plans on a batch (before its first solve)."""
    b.set_class_plans([{k: p[k] for k in ("n_hi", "block", "chunk", "placement")} for p in plans])
