"""Comparators for the batched persistent launch.

The paper compares its one-kernel team design against a naive per-problem
launch loop and against several such loops sharing the GPU through NVIDIA's
multi-process service (section IV).  On MI355X the equivalent of the latter
is several host threads, each driving the per-problem launch loop
(dr_solve_loop: a few kernels per pass and a host round trip for the stop
test) on its own HIP stream, so that their passes overlap on the device.
Every problem's result is the same as in a single loop.
"""
from __future__ import annotations

import threading
import time
from typing import List

import numpy as np

from . import dr


def multistream_loop(batch, n_streams: int, **opts) -> dict:
    """Solves every network of `batch` with the per-problem launch loop on
    `n_streams` host threads, each with its own stream and its own share of
    the networks (round robin).  Returns the wall time and the per-network
    results in batch order."""
    import torch
    n_streams = max(1, min(int(n_streams), len(batch)))
    shares: List[List[int]] = [list(range(k, len(batch), n_streams)) for k in range(n_streams)]
    streams = [torch.cuda.Stream() for _ in shares]
    batches = [dr.DRBatch(batch.subset(ids), stream=st.cuda_stream, **opts)
               for ids, st in zip(shares, streams)]
    errors: List[BaseException] = []
    start = threading.Barrier(n_streams + 1)

    def work(b):
        try:
            start.wait()
            b.solve_loop()
        except BaseException as e:  # reported after join
            errors.append(e)

    threads = [threading.Thread(target=work, args=(b,)) for b in batches]
    for t in threads:
        t.start()
    start.wait()
    t0 = time.perf_counter()
    for t in threads:
        t.join()
    wall = time.perf_counter() - t0
    if errors:
        raise errors[0]
    P = len(batch)
    out = dict(wall_s=wall, n_streams=n_streams, sigma=np.zeros((P, 3, 3)),
               iters=np.zeros(P, np.int64), result=np.zeros(P, np.int32))
    for ids, b in zip(shares, batches):
        r = b.results()
        out["sigma"][ids] = r["sigma"]
        out["iters"][ids] = r["iters"]
        out["result"][ids] = r["result"]
        b.close()
    M = np.array([n.n_fibers for n in batch.nets], np.float64)
    out["updates"] = float((M * out["iters"]).sum())
    out["updates_per_s"] = out["updates"] / wall
    return out
