"""Launch-shape autotuner for batches of uneven size.

The paper runs every sub-problem with one fixed team size (section IV); on
gfx950 the best shape depends on the node count: how many nodes each lane
holds, whether the nodal state fits in LDS, how far ahead the gather loads,
and how many workgroups share a compute unit.  The tuner splits a batch's
node-count range into buckets and picks one plan (block, chunk, placement)
per bucket for dr_set_class_plans.

Plans are scored on the whole batch, because the size classes of a launch
run concurrently and compete for compute units and memory bandwidth: a plan
that is fastest for a bucket alone can slow the batch down.  Starting from
the library's automatic plans, the tuner visits the buckets in order of the
fibers they carry and, for each, keeps the candidate that shortens a
fixed-pass launch of the whole batch by at least 2 %.  The result is then
confirmed against the library's default split (no plans: one class for the
LDS-resident sizes, one for the rest) on launches of the pass count the
plans are for (by default ten times the search's: short launches overweight
set-up, and how the classes' workgroups fall into rounds on the compute
units changes with the launch length) and kept only if it is faster there
too; otherwise the tuner returns no plans.  Every launch shape
computes the same per-node arithmetic in the same order, so a candidate must
also reproduce the incumbent's pass counts exactly; one that does not is
rejected.

Results are cached in memory and, if a path is given, in a JSON file keyed by
device architecture, compute-unit count, precision, pass count and the
batch's bucket histogram.
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
    block: int      # 0 = automatic
    chunk: int      # 0 = automatic
    placement: int  # a dr_placement value

    def as_dict(self, n_hi: int) -> dict:
        return dict(n_hi=int(n_hi), block=self.block, chunk=self.chunk, placement=self.placement)


AUTO = Plan(0, 0, dr.DR_PLACE_AUTO)


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
        # global placement with 256 lanes runs chunks of 1 only
        for ch in ((1,) if blk == 256 else CHUNKS):
            out.append(Plan(blk, ch, dr.DR_PLACE_GLOBAL))
    return out


def device_key(precision: int) -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return f"{getattr(p, 'gcnArchName', p.name)}|cu{p.multi_processor_count}|prec{precision}"


class BatchTimer:
    """Times launches of one batch, every problem started afresh and run for
    a fixed number of passes, under given class plans."""

    def __init__(self, batch, *, precision: int, reps: int,
                 clock: Callable[[], float] = time.perf_counter):
        self.batch = batch
        self.b = dr.DRBatch(batch, tol=1e-300, max_iter=2 ** 62, precision=precision)
        self.ids = np.arange(len(batch), dtype=np.int32)
        self.starts = np.full(len(batch), dr.DR_START_AFFINE, np.int32)
        self.reps = reps
        self.clock = clock

    def _launch(self, passes: int):
        self.b.advance(self.ids, self.starts, passes, F=self.batch.F)
        self.b.sync()

    def __call__(self, plans: List[dict], passes: int) -> Optional[Tuple[float, np.ndarray]]:
        """(median seconds per launch, pass counts), or None when the library
        rejects the plans."""
        try:
            self.b.set_class_plans(plans)
        except dr.DrError as e:
            if e.status == dr.DR_E_INVALID:
                return None
            raise
        self._launch(passes)  # warm-up (loads the shapes' kernels)
        ts = []
        for _ in range(self.reps):
            t0 = self.clock()
            self._launch(passes)
            ts.append(self.clock() - t0)
        return float(np.median(ts)), self.b.query(self.ids)["iters"].copy()

    def close(self):
        self.b.close()


class Tuner:
    def __init__(self, *, edges: Sequence[int] = DEFAULT_EDGES, passes: int = 300, reps: int = 1,
                 confirm_passes: Optional[int] = None, cache_path: Optional[str] = None,
                 timer_factory: Optional[Callable] = None,
                 key: Optional[Callable[[int], str]] = None,
                 log: Callable[[str], None] = lambda s: None):
        self.edges = tuple(edges)
        self.passes = int(passes)
        self.confirm_passes = int(confirm_passes or 10 * passes)
        self.reps = int(reps)
        self.cache_path = cache_path
        self.timer_factory = timer_factory or (
            lambda batch, precision: BatchTimer(batch, precision=precision, reps=self.reps))
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
        """Class plans (ascending n_hi) for dr_set_class_plans; block, chunk
        and placement 0 mean the library's automatic choice; an empty list
        keeps the library's default split."""
        sizes = np.array([n.n_nodes for n in batch.nets])
        fibers = np.array([n.n_fibers for n in batch.nets])
        bks = buckets(sizes, self.edges)
        ckey = (f"{self.key(precision)}|K{self.passes}/{self.confirm_passes}|" +
                ",".join(f"{lo}-{hi}:{len(idx)}" for lo, hi, idx in bks))
        if ckey in self.cache:
            return [dict(p) for p in self.cache[ckey]["plans"]]
        timer = self.timer_factory(batch, precision)
        try:
            his = [hi for _, hi, _ in bks]
            cur = [AUTO] * len(bks)

            def as_plans(pl):
                return [p.as_dict(h) for p, h in zip(pl, his)]
            res = timer(as_plans(cur), self.passes)
            if res is None:
                raise dr.DrError(dr.DR_E_INVALID, "the automatic plans were rejected")
            t_best, iters_ref = res
            t_auto = t_best
            self.log(f"automatic plans: {t_best * 1e3:.2f} ms")
            order = sorted(range(len(bks)), key=lambda k: -int(fibers[bks[k][2]].sum()))
            for k in order:
                lo, hi, idx = bks[k]
                for cand in candidates(int(sizes[idx].max())):
                    trial = list(cur)
                    trial[k] = cand
                    res = timer(as_plans(trial), self.passes)
                    if res is None:
                        continue
                    t, iters = res
                    if not np.array_equal(iters, iters_ref):
                        self.log(f"bucket ({lo},{hi}] {cand}: pass counts differ, rejected")
                        continue
                    self.log(f"bucket ({lo},{hi}] {cand}: {t * 1e3:.2f} ms")
                    if t < 0.98 * t_best:
                        cur, t_best = trial, t
            plans = as_plans(cur)
            long = self.confirm_passes
            t_tuned = timer(plans, long)[0]
            t_default = timer([], long)[0]
            confirm = dict(passes=long, ms_tuned=t_tuned * 1e3, ms_default=t_default * 1e3)
            self.log(f"confirm at {long} passes: tuned {t_tuned * 1e3:.1f} ms, default split "
                     f"{t_default * 1e3:.1f} ms")
            if not t_tuned < 0.98 * t_default:
                plans = []
            self.cache[ckey] = dict(plans=plans, ms=t_best * 1e3, ms_automatic=t_auto * 1e3,
                                    confirm=confirm)
            self._save()
            return [dict(p) for p in plans]
        finally:
            timer.close()


def apply(b: "dr.DRBatch", plans: List[dict]):
    """Install tuned class plans on a batch."""
    b.set_class_plans([{k: p[k] for k in ("n_hi", "block", "chunk", "placement")} for p in plans])
