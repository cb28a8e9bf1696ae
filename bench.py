#!/usr/bin/env python3
"""Benchmark of batched dynamic relaxation on one MI355X.

Workload (default): 256 random kNN fiber networks, node counts uniform in
1000..5000, FP64, F = I + sym U(+-0.01), relative residual 1e-8, damping
1e-4, solved by one persistent launch per step through the C ABI.  A step
is one solve of every network to convergence (set-up, DR loop, stress) with
the stress read back to the host.

Metric: fiber-element updates/s = sum_p fibers_p * passes_p / wall time.
Beside it: the same networks' per-problem launch loop (a sample solved to
convergence), the FP32-state solve of the batch with its per-network stress
error, the continuous-batching serving loop over the batch as a resident
pool (p50/p99 latency at three offered rates), and the CPU oracle (a bounded
sample, all host threads).  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of one fiber-element update (one DR pass over one fiber,
# with its share of the per-node work), counted once per fiber:
#   fiber: d (3), l^2 (5), k (l^2 - L^2) / l (4), force on both ends (9)  = 21
#   node (x0.47 nodes per fiber): update x (6), damped acceleration (6),
#   two half velocity updates (12), |g|^2 (6), m |v|^2 (7)                 = 37 -> 17
FLOP_PER_UPDATE = 38.0
# Compulsory HBM bytes per fiber-update if the nodal state lived in HBM
# (FP64: per free node u, v read+write 96 B; per node X 24 B, 1/m 8 B, row
# pointer 4 B; per fiber 2 incidences x (4 B index + 16 B constants)).
BYTES_PER_UPDATE = 104.0
# The same for the FP32 state (per fiber 2 incidences x (4 B index + 16 B of
# FP32 reference vector and constant); per free node the FP32 state with its
# compensation terms and the velocity read and written; per node 1/m and the
# row pointer): about 75 B per fiber-update.
BYTES_PER_UPDATE_FP32 = 75.0
PEAK_FP64_VECTOR = 78.6e12
PEAK_HBM = 8.0e12

# Bytes one launch moves beyond L2 (HBM and Infinity Cache), from rocprofv3
# FETCH_SIZE and WRITE_SIZE runs of this benchmark scaled by what the same
# counters read for a plain copy of known size (profiles/ holds the summary
# and the commands).  Valid only for the kernel source it was measured on:
# any change to the kernels makes the figure null until it is measured again.
MEASURED_TRAFFIC = {
    # profiles/k_dr_reg_uniform256_fp64.md: FETCH 7.15131e9 KiB x 1.9998 + WRITE 18354.5 KiB x 1.0
    "uniform": {"kernels": "b0d5014e1253bb79", "bytes_per_launch": 1.4644e13},
    # profiles/k_dr_reg_uniform256_fp32.md: FETCH 6.94796e9 KiB x 1.9998 + WRITE 18357.3 KiB x 1.0
    "uniform32": {"kernels": "b0d5014e1253bb79", "bytes_per_launch": 1.4228e13},
    # profiles/k_dr_glb_uneven1024_fp64.md: both DR kernels and the stress of one 20 000-pass
    # launch (default plans), per launch of the two the run makes
    "uneven": {"kernels": "b0d5014e1253bb79", "bytes_per_launch": 4.4016e13},
}


def kernels_digest():
    """Digest of every device source (the kernels, their templates and the
    data layout), in file-name order."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2305_07030_amd", "csrc")
    for p in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.h"))):
        with open(p, "rb") as f:
            h.update(os.path.basename(p).encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def traffic_for(workload):
    t = MEASURED_TRAFFIC.get(workload)
    if t is None or t["kernels"] != kernels_digest():
        return None
    return t["bytes_per_launch"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def host_cpu():
    """The host's CPU model and counts: os.cpu_count(), the CPUs this process
    may run on, and the share used (the CPUs this process may use, at most 16:
    the GPU hosts give each GPU's jobs a share of 16 cores)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    return {"model": model, "nproc": os.cpu_count(), "affinity": affinity,
            "used": max(1, min(16, affinity))}


def cpu_baseline(batch, beta, tol, target_s=15.0):
    """The oracle, untuned, on a bounded sample: the first C networks, a fixed
    number of DR passes each, one network per thread (C = the host's CPU
    share, see host_cpu)."""
    import numpy as np

    import oracle as O
    from concurrent.futures import ThreadPoolExecutor
    O.build(force=False)
    cpu = host_cpu()
    C = cpu["used"]
    sub = batch.subset(range(min(C, len(batch))))
    # calibrate the pass count on one network
    t = time.perf_counter()
    O.solve(sub.nets[0], sub.F[0], tol=1e-300, max_iter=500, beta=beta, dt_safety=0.9)
    per_pass = (time.perf_counter() - t) / 500 / sub.nets[0].n_fibers
    mean_m = np.mean([n.n_fibers for n in sub.nets])
    passes = int(max(1000, min(200000, target_s / (per_pass * mean_m))))
    t = time.perf_counter()
    with ThreadPoolExecutor(max_workers=C) as ex:
        res = list(ex.map(lambda i: O.solve(sub.nets[i], sub.F[i], tol=1e-300, max_iter=passes,
                                            beta=beta, dt_safety=0.9), range(len(sub))))
    wall = time.perf_counter() - t
    upd = sum(n.n_fibers * r.iters for n, r in zip(sub.nets, res))
    return {"value": upd / wall, "unit": "fiber-updates/s", "cores": C, "kind": "oracle",
            "sample": f"first {len(sub)} networks of the batch, {passes} DR passes each "
                      f"(fixed pass count), one network per thread, {wall:.1f}s wall",
            "host": cpu}


def loop_baseline(batch, beta, tol, stream, quantiles=(0.0, 0.25, 0.5, 0.75, 1.0)):
    """The per-problem launch loop (the paper's naive design) on a stratified
    sample: the networks at the given quantiles of the node count, each
    solved to convergence (same tolerance and iteration as the batched
    launch); rate = sum M n / sum t."""
    import numpy as np

    from paper_2305_07030_amd import dr
    sizes = np.array([n.n_nodes for n in batch.nets])
    order = np.argsort(sizes, kind="stable")
    pick = sorted({int(order[min(len(order) - 1, int(round(q * (len(order) - 1))))]) for q in quantiles})
    upd = wall = 0.0
    rows = []
    for i in pick:
        lb = dr.DRBatch(batch.subset([i]), tol=tol, damping=beta, dt_safety=0.9, stream=stream.cuda_stream)
        t = time.perf_counter()
        lb.solve_loop()
        r = lb.results()
        dt = time.perf_counter() - t
        lb.close()
        m = batch.nets[i].n_fibers * int(r["iters"][0])
        upd += m
        wall += dt
        rows.append({"network": i, "nodes": int(sizes[i]), "passes": int(r["iters"][0]),
                     "seconds": round(dt, 3), "us_per_pass": round(dt / int(r["iters"][0]) * 1e6, 2)})
        log(f"loop baseline: network {i} (N={sizes[i]}) {int(r['iters'][0])} passes in {dt:.2f}s")
    return {"value": upd / wall, "unit": "fiber-updates/s",
            "sample": f"networks at node-count quantiles {list(quantiles)} solved to convergence by the "
                      f"per-problem launch loop; rate = sum M n / sum t",
            "networks": rows}


def ceilings():
    """Measured copy bandwidths: a buffer pair that fits in the 256 MB
    Infinity Cache (MALL) copied repeatedly, and one that does not (HBM)."""
    import torch
    out = {}
    for name, mib, reps in (("mall_copy", 48, 200), ("hbm_copy", 2048, 10)):
        x = torch.ones(mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        s = e0.elapsed_time(e1) / 1e3
        out[name + "_GBps"] = 2 * mib * (1 << 20) * reps / s / 1e9
        out[name + "_bytes"] = 2 * mib * (1 << 20)
        del x, y
    log("ceilings:", out)
    return out


# Damping of the FP32-state workloads: the FP32 residual floor falls steeply
# with the damping (median floor on 64 networks of the 256-network batch,
# MI355X: 1.0e-3 at 1e-4, 2.3e-4 at 3e-4, 3.5e-5 at 1e-3, 5.0e-6 at 3e-3,
# 1.2e-6 at 1e-2, 1.0e-6 at 3e-2), and only from about 3e-2 on do most
# solves reach tol 1e-6.
FP32_DAMPING = 3e-2


def fp32_leg(batch, stream, beta=FP32_DAMPING):
    """The same networks with FP32 nodal state and force gather (FP64 norms
    and stress), tol 1e-6 with a 50 000-pass stall guard, against an FP64
    solve of the same iteration (same damping, tol 1e-8).  FP32 rounding is
    re-injected every pass and the lightly damped modes integrate it, so the
    residual it can reach falls steeply with the damping (FP32_DAMPING); the
    FP64 workload's 1e-4 would leave it near rho ~ 1e-3."""
    import numpy as np
    import torch

    from paper_2305_07030_amd import dr
    M = np.array([n.n_fibers for n in batch.nets], np.float64)
    Fd = torch.tensor(batch.F.reshape(-1, 9), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    b64 = dr.DRBatch(batch, tol=1e-8, damping=beta, dt_safety=0.9, stream=stream.cuda_stream)
    t = time.perf_counter()
    b64.solve_device(Fd)
    r64 = b64.results()
    wall64 = time.perf_counter() - t
    b64.close()
    b = dr.DRBatch(batch, tol=1e-6, damping=beta, dt_safety=0.9, precision=dr.DR_FP32,
                   stall_window=50_000, stream=stream.cuda_stream)
    b.solve_device(Fd)
    b.results()
    torch.cuda.synchronize()
    t = time.perf_counter()
    b.solve_device(Fd)
    r = b.results()
    wall = time.perf_counter() - t
    s32 = r["sigma"].reshape(len(batch), 9)
    s64 = r64["sigma"].reshape(len(batch), 9)
    err = np.linalg.norm(s32 - s64, axis=1) / np.linalg.norm(s64, axis=1)
    upd = float((M * r["iters"]).sum())
    b.close()
    return {"value": upd / wall, "unit": "fiber-updates/s", "wall_s": wall, "damping": beta,
            "converged": int((r["result"] == dr.DR_CONVERGED).sum()),
            "stalled": int((r["result"] == dr.DR_STALLED).sum()),
            "rho_median": float(np.median(r["rho"])), "rho_max": float(r["rho"].max()),
            "passes_median": int(np.median(r["iters"])), "passes_max": int(r["iters"].max()),
            "fp64_reference": {"wall_s": wall64, "tol": 1e-8,
                               "converged": int((r64["result"] == dr.DR_CONVERGED).sum()),
                               "passes_median": int(np.median(r64["iters"])),
                               "passes_max": int(r64["iters"].max())},
            "sigma_rel_err_vs_fp64": {"median": float(np.median(err)),
                                      "p99": float(np.percentile(err, 99)),
                                      "max": float(err.max())},
            "per_network_sigma_rel_err": [float(x) for x in err]}


def multistream_leg(batch, beta, n_nets=16, passes=20000):
    """The per-problem launch loop run by 1, 4 and 16 host threads, each on its
    own stream (the multi-process-service comparison of the paper, section
    IV): the first n_nets networks, a fixed pass count each."""
    from paper_2305_07030_amd import compare as CMP
    sub = batch.subset(range(n_nets))
    out = {"sample": f"first {n_nets} networks, {passes} passes each (fixed pass count)",
           "unit": "fiber-updates/s"}
    for n in (1, 4, 16):
        r = CMP.multistream_loop(sub, n, tol=1e-300, max_iter=passes, damping=beta, dt_safety=0.9)
        out[f"streams_{n}"] = r["updates_per_s"]
        log(f"loop on {n} streams: {r['updates_per_s']:.3e} updates/s ({r['wall_s']:.2f}s)")
    # the paper's zero + atomic-scatter force kernel in the same loop, one network
    from paper_2305_07030_amd import dr
    one = batch.subset([0])
    for scatter in (False, True):
        b = dr.DRBatch(one, tol=1e-300, max_iter=passes, damping=beta, dt_safety=0.9)
        t = time.perf_counter()
        b.solve_loop(scatter=scatter)
        b.results()
        wall = time.perf_counter() - t
        b.close()
        out["scatter_us_per_pass" if scatter else "gather_us_per_pass"] = wall / passes * 1e6
    log("loop pass times (us): gather", out["gather_us_per_pass"], "scatter", out["scatter_us_per_pass"])
    return out


def serving_leg(pool_batch, n_closed=192, rates=(0.5, 0.8, 0.95), n_warm=16, n_meas=64):
    """The serving configuration at its own size, shortened: the 4096-network
    pool (FP64, tol 1e-8, 384 MiB of running state) through the library's
    pool, a cold closed loop for the saturated rate and short open-loop runs
    at fractions of it (pool_run; `--workload pool` runs the long form)."""
    r = pool_run(pool_batch, False, 384 << 20, n_closed, list(rates), n_warm, n_meas, 90.0, drain_s=20.0)
    r["counts"] = f"closed loop {n_closed} requests, open loop {n_warm} + {n_meas} per rate"
    return r


def copy_calibration(mib):
    """One plain copy of `mib` MiB (reads and writes it once), whose traffic
    counters scale the DR kernels' (the same counters read for known bytes)."""
    if not mib:
        return
    import torch
    x = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    log(f"copy calibration: {mib} MiB read, {mib} MiB written")
    del x, y


def _pool_part(a):
    from paper_2305_07030_amd import inputs as I
    P, lo, hi = a
    return I.config_pool(P, idx=list(range(lo, hi)))


def make_pool_batch(P):
    """The serving pool's networks (N log-uniform in [1000, 33000], seed base
    5), generated in worker processes: call before this process touches the
    GPU."""
    from concurrent.futures import ProcessPoolExecutor

    import numpy as np

    from paper_2305_07030_amd import inputs as I
    t = time.perf_counter()
    cuts = np.linspace(0, P, 17).astype(int)
    with ProcessPoolExecutor(16) as ex:
        parts = list(ex.map(_pool_part, [(P, int(a), int(b)) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]))
    batch = I.Batch([n for b in parts for n in b.nets], np.concatenate([b.F for b in parts]))
    log(f"pool: {P} networks, {batch.total_nodes} nodes, {batch.total_fibers} fibers, generated in "
        f"{time.perf_counter() - t:.1f}s")
    return batch


def pool_run(batch, fp32, budget, n_requests, rates, warm, measure, open_limit, drain_s=60.0):
    """The library's pool (dr_pool_*) over `batch` with a running-state budget
    below capacity, so that admission binds.  Closed loop: n_requests
    requests of the arrival stream (pool ids and F walk) queued at once on a
    cold pool (a network's first request starts from the affine field), run
    until 90 % are done: the saturated rate is the completions between the
    10th and the 90th percentile times.  Then open-loop Poisson arrivals at
    the given fractions of it (warm + measure requests each).  Latency =
    enqueue (arrival) to sigma on the host."""
    import numpy as np
    import torch

    from paper_2305_07030_amd import dr
    from paper_2305_07030_amd import serve as SV
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    P = len(batch)
    M = np.array([n.n_fibers for n in batch.nets])
    # FP32 state: tol 1e-6 at the damping where its residual floor lies below
    # it (see fp32_leg), the stall guard on
    popt = (dict(tol=1e-6, damping=FP32_DAMPING, precision=dr.DR_FP32, stall_window=50_000) if fp32
            else dict(tol=1e-8, damping=1e-4))
    t = time.perf_counter()
    pool = dr.Pool(batch, state_budget_bytes=budget, max_slots=256, tick_passes=4000, dt_safety=0.9,
                   **popt)
    log(f"pool created in {time.perf_counter() - t:.1f}s")
    stream = SV.RequestStream(batch.F, 0.0, 0.002, seed=50)
    reqs = [stream.make(0.0) for _ in range(n_requests)]
    t0 = time.perf_counter()
    for r in reqs:
        pool.submit(r.net, r.F, r.rid)
    lat, res, its, nets, polls = [], [], [], [], 0
    tick_s, tick_flight = [], []
    t_last = t0
    target = int(np.ceil(0.9 * n_requests))
    while len(lat) < target:
        st = pool.status()
        flight = st["in_flight"] + min(st["queued"], 256)
        tp = time.perf_counter()
        out = pool.poll()
        polls += 1
        now = time.perf_counter()
        tick_s.append(now - tp)
        tick_flight.append(flight)
        lat += [now - t0] * len(out["tags"])
        res += out["result"].tolist()
        its += out["iters"].tolist()
        nets += out["ids"].tolist()
        if now - t_last > 20:
            st = pool.status()
            log(f"t={now - t0:.0f}s: {len(lat)} done, {st['in_flight']} in flight, {st['queued']} queued, "
                f"{st['state_bytes'] >> 20} MiB of state")
            t_last = now
    wall = time.perf_counter() - t0
    lat = np.array(lat)
    upd = float(sum(M[n] * i for n, i in zip(nets, its)))
    t10, t90 = np.percentile(lat, 10), np.percentile(lat, 90)
    sat = 0.8 * len(lat) / max(t90 - t10, 1e-9) * (n_requests / len(lat))
    seen = set(nets)
    log(f"closed loop: saturated {sat:.3f} solves/s, first {len(lat)} of {n_requests} done in {wall:.1f}s, "
        f"p50 {np.percentile(lat, 50):.1f}s")
    open_loop = []
    tag0 = len(reqs)
    for frac in rates:
        r = pool_open_loop(pool, stream, frac * sat, warm, measure, open_limit, seen, tag0, drain_s)
        tag0 += warm + measure
        r["offered_fraction"] = frac
        open_loop.append(r)
        log(f"open loop at {frac} x saturation: {r}")
    pool.close()
    prec = "FP32 state, tol 1e-6, damping %g" % FP32_DAMPING if fp32 else "FP64, tol 1e-8, damping 1e-4"
    return {"pool": f"{P} kNN(k=3) networks, N log-uniform [1000, 33000], F walk sym U(+-0.002), {prec}, "
                    f"cold pool",
            "state_budget_bytes": budget, "max_slots": 256, "tick_passes": 4000,
            "ticks": "fixed length, budgets from dr_batch_pass_costs",
            "saturated_solves_per_s": sat,
            "closed_loop": {"requests": n_requests, "measured_until": len(lat), "wall_s": wall, "polls": polls,
                            "p50_s": float(np.percentile(lat, 50)), "fiber_updates_per_s": upd / wall,
                            "poll_s": {"p10": float(np.percentile(tick_s, 10)),
                                       "p50": float(np.percentile(tick_s, 50)),
                                       "p90": float(np.percentile(tick_s, 90)), "max": float(np.max(tick_s))},
                            "in_flight_at_poll": {"p10": float(np.percentile(tick_flight, 10)),
                                                  "p50": float(np.percentile(tick_flight, 50)),
                                                  "p90": float(np.percentile(tick_flight, 90))},
                            "results": {str(k): int(sum(r == k for r in res)) for k in sorted(set(res))}},
            "open_loop": open_loop}


def pool_main(args):
    """The serving configuration at its own size (--pool-size networks),
    closed loop then open-loop rates (pool_run), as its own line."""
    batch = make_pool_batch(args.pool_size)
    rates = [float(x) for x in args.rates.split(",")] if args.rates else []
    r = pool_run(batch, args.precision == "fp32", args.state_budget_mib << 20, args.requests, rates,
                 args.warm, args.measure, args.open_limit)
    line = {"metric": "solves/s (serving pool, saturated)", "value": r["saturated_solves_per_s"],
            "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
            "dtype": "f32" if args.precision == "fp32" else "f64", "data": "synthetic",
            "config": {"workload": r["pool"], "requests": args.requests}, **r}
    print(json.dumps(line), flush=True)


def pool_open_loop(pool, stream, rate, n_warm, n_meas, max_wall, seen, tag0, drain_s=60.0):
    """Poisson arrivals at `rate` (wall clock) into the library's pool; each
    poll submits the requests that have arrived, runs one tick and collects
    the finished ones.  Latency = arrival to the result on the host; the
    first n_warm requests are not measured.  `seen`: networks solved before
    (their requests start warm); updated.  Tags start at tag0 (a result of an
    earlier run that finishes during this one is not counted); the run drains
    its own requests for at most drain_s after its last arrival."""
    import numpy as np

    from paper_2305_07030_amd import dr
    stream.rate = rate
    t0 = time.perf_counter()
    t_next = t0 + stream.next_gap()
    arrival, lat, res = {}, [], []
    issued = done = warm = 0
    total = n_warm + n_meas
    t_log = t0
    while done < total and time.perf_counter() - t0 < max_wall:
        now = time.perf_counter()
        if now - t_log > 20:
            st = pool.status()
            log(f"open loop {rate:.2f}/s: t={now - t0:.0f}s, {issued} issued, {done} done, "
                f"{st['in_flight']} in flight, {st['queued']} queued")
            t_log = now
        while issued < total and t_next <= now:
            r = stream.make(t_next)
            if issued >= n_warm and r.net in seen:
                warm += 1
            seen.add(r.net)
            pool.submit(r.net, r.F, tag0 + issued)
            arrival[tag0 + issued] = t_next
            issued += 1
            t_next += stream.next_gap()
        st = pool.status()
        if st["queued"] == 0 and st["in_flight"] == 0 and st["completed"] == 0:
            time.sleep(max(0.0, min(t_next - time.perf_counter(), 0.05)))
            continue
        out = pool.poll()
        now = time.perf_counter()
        for tag, rr in zip(out["tags"], out["result"]):
            if int(tag) not in arrival:
                continue  # a request of an earlier run
            done += 1
            if tag >= tag0 + n_warm:
                lat.append(now - arrival[int(tag)])
                res.append(int(rr))
        if issued >= total and now - t_next > drain_s:
            break
    wall = time.perf_counter() - t0
    lat = np.array(lat) if lat else np.zeros(1)
    return {"offered_per_s": rate, "measured": len(res), "measured_warm_starts": warm, "issued": issued,
            "completed": done,
            "throughput_per_s": done / wall, "p50_s": float(np.percentile(lat, 50)),
            "p90_s": float(np.percentile(lat, 90)), "p99_s": float(np.percentile(lat, 99)), "wall_s": wall,
            "converged": int(sum(r == dr.DR_CONVERGED for r in res)),
            "results": {str(k): int(sum(r == k for r in res)) for k in sorted(set(res))}}


def resident_main(args):
    """Bytes beyond L2 of the global-placement kernel against the number of
    problems resident at once: `--copies` copies of one 16 000-node kNN
    network (workgroups are dealt to the 8 XCDs round robin, so copies / 8
    share one XCD's 4 MB L2), global placement, `--passes` fixed passes."""
    import numpy as np
    import torch

    from paper_2305_07030_amd import dr
    from paper_2305_07030_amd import inputs as I
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    rng = np.random.default_rng(7)
    net = I.draw_network(rng, 16000)
    F = I.sym_perturbed_F(rng, 0.02)
    C, K = args.copies, args.passes
    batch = I.Batch([net] * C, np.stack([F] * C))
    b = dr.DRBatch(batch, tol=1e-300, max_iter=K, damping=1e-4, dt_safety=0.9, placement=dr.DR_PLACE_GLOBAL)
    walls = []
    for _ in range(2):
        t = time.perf_counter()
        b.solve()
        r = b.results()
        walls.append(time.perf_counter() - t)
    b.close()
    upd = float(C) * net.n_fibers * K
    line = {"metric": "fiber-element updates/s (global placement, resident copies)", "value": upd / walls[-1],
            "unit": "fiber-updates/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": f"{C} copies of one 16000-node kNN(k=3) network, global placement, "
                                   f"{K} passes", "copies": C, "nodes": net.n_nodes, "fibers": net.n_fibers,
                       "passes": K},
            "us_per_pass": walls[-1] / K * 1e6, "iters_min": int(r["iters"].min())}
    print(json.dumps(line), flush=True)


def uneven_main(args):
    """The 1024-network batch with node counts log-uniform in [2000, 33000]:
    launch shapes tuned per size bucket, the solve step captured in a HIP
    graph; a step is one graph launch making a fixed number of passes on
    every network (plus the stress), timed against the untuned default plans.
    With --converge the batch is then solved to convergence in budgeted
    launches (progress printed after each)."""
    import numpy as np
    import torch

    from paper_2305_07030_amd import dr
    from paper_2305_07030_amd import inputs as I
    from paper_2305_07030_amd import tune as T

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dr.load()
    t = time.perf_counter()
    batch = I.config_uneven_batch(1024)
    M = np.array([n.n_fibers for n in batch.nets], np.float64)
    N = np.array([n.n_nodes for n in batch.nets])
    log(f"generated 1024 networks, {int(N.sum())} nodes, {int(M.sum())} fibers in "
        f"{time.perf_counter() - t:.1f}s")
    beta, K = 1e-4, args.passes
    wl = ("1024 kNN(k=3) fiber networks, N = round(exp U(ln 2000, ln 33000)), "
          "F = I + sym U(+-0.02), FP64")
    copy_calibration(args.copy_mib)
    tuner = T.Tuner(passes=300, reps=1, confirm_passes=K, log=lambda m: log("tune:", m))
    t = time.perf_counter()
    plans = [] if args.no_tune else tuner.tune(batch)
    tune_s = time.perf_counter() - t
    log(f"tuned in {tune_s:.1f}s:", [{k: p[k] for k in ("n_hi", "block", "chunk", "placement")}
                                     for p in plans])
    stream = torch.cuda.Stream()
    Fd = torch.tensor(batch.F.reshape(-1, 9), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()  # F is in HBM before the batch stream uses it

    def timed(b, use_graph, label):
        if use_graph:
            b.graph_capture(Fd)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        for w in range(args.warmup):
            b.graph_launch() if use_graph else b.solve_device(Fd)
            b.results()
            log(f"{label} warmup {w} done")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            ev[k][0].record(stream)
            b.graph_launch() if use_graph else b.solve_device(Fd)
            ev[k][1].record(stream)
            r = b.results()
            log(f"{label} step {k}: {ev[k][0].elapsed_time(ev[k][1]):.1f} ms")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # every network makes the K passes unless it diverges (NONFINITE) first
        done = (r["result"] == dr.DR_MAX_ITER) | (r["result"] == dr.DR_NONFINITE)
        assert done.all() and (r["iters"][r["result"] == dr.DR_MAX_ITER] == K).all()
        upd = float((M * r["iters"]).sum())
        kern = sum(a.elapsed_time(e) for a, e in ev) / 1e3 / args.steps
        return upd * args.steps / wall, wall / args.steps, kern, upd, r

    with torch.cuda.stream(stream):
        bt = dr.DRBatch(batch, tol=1e-300, max_iter=K, damping=beta, dt_safety=0.9,
                        stream=stream.cuda_stream)
        T.apply(bt, plans)
        classes = bt.classes()
        v_tuned, step_s, kern_s, upd, r = timed(bt, True, "tuned+graph")
        bt.close()
        bd = dr.DRBatch(batch, tol=1e-300, max_iter=K, damping=beta, dt_safety=0.9,
                        stream=stream.cuda_stream)
        default_classes = bd.classes()
        v_default, dstep_s, _, _, _ = timed(bd, False, "default")
        bd.close()
    n_div = int((r["result"] == dr.DR_NONFINITE).sum())
    out = {
        "metric": "fiber-element updates/s (batched persistent launch, fixed pass count)",
        "value": v_tuned, "unit": "fiber-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": step_s * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl, "networks": 1024, "nodes": int(N.sum()), "fibers": int(M.sum()),
                   "passes_per_step": K, "diverged_before_K": n_div, "damping": beta,
                   "dt_safety": 0.9,
                   "plans": [{k: p[k] for k in ("n_hi", "block", "chunk", "placement")} for p in plans],
                   "classes": classes, "tuning_s": tune_s},
        "default_plans": {"value": v_default, "ms_per_step": dstep_s * 1e3,
                          "classes": default_classes},
        "roofline": {"bound": "hbm", "achieved": BYTES_PER_UPDATE * upd / kern_s / 1e9,
                     "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                     "frac": BYTES_PER_UPDATE * upd / kern_s / PEAK_HBM,
                     "traffic": traffic_for("uneven") if K == 20000 and not plans else None,
                     "kernel": "k_dr_glb with k_dr_reg (the two size classes of one launch, run "
                               "concurrently; the networks above the LDS limit carry most fibers)",
                     "kernel_ms": kern_s * 1e3, "bytes_per_update": BYTES_PER_UPDATE},
    }
    if args.converge:
        out["converge"] = uneven_converge(batch, plans, beta, M, args.converge_limit, args.tail_at,
                                          args.tail_group)
    print(json.dumps(out), flush=True)


def uneven_leg(passes=20000):
    """The 1024-network workload (N log-uniform in [2000, 33000]) beside the
    main line: one graph-captured step of `passes` passes on every network
    with the library's default plans (after one untimed step), timed with
    HIP events on the batch stream."""
    import numpy as np
    import torch

    from paper_2305_07030_amd import dr
    from paper_2305_07030_amd import inputs as I
    t = time.perf_counter()
    batch = I.config_uneven_batch(1024)
    M = np.array([n.n_fibers for n in batch.nets], np.float64)
    gen = time.perf_counter() - t
    stream = torch.cuda.Stream()
    Fd = torch.tensor(batch.F.reshape(-1, 9), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        b = dr.DRBatch(batch, tol=1e-300, max_iter=passes, damping=1e-4, dt_safety=0.9,
                       stream=stream.cuda_stream)
        b.graph_capture(Fd)
        b.graph_launch()
        b.results()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        b.graph_launch()
        e1.record(stream)
        r = b.results()
        wall = time.perf_counter() - t0
        classes = b.classes()
        b.close()
    upd = float((M * r["iters"]).sum())
    kern = e0.elapsed_time(e1) / 1e3
    out = {"workload": "1024 kNN(k=3) fiber networks, N = round(exp U(ln 2000, ln 33000)), "
                       f"F = I + sym U(+-0.02), FP64, {passes} passes per network (fixed pass count), "
                       "graph-captured step, default plans",
           "value": upd / wall, "unit": "fiber-updates/s", "step_s": wall, "kernel_s": kern,
           "nonfinite_before_K": int((r["result"] == dr.DR_NONFINITE).sum()),
           "hbm_equivalent_frac": BYTES_PER_UPDATE * upd / kern / PEAK_HBM,
           "classes": classes, "generation_s": gen}
    log("uneven leg:", out)
    return out


def uneven_converge(batch, plans, beta, M, limit_s, tail_at=0, tail_group=0):
    """Every network to tol 1e-8 (max 2e6 passes) in launches of at most
    100 000 passes each (with tail_at > 0 the last tail_at running problems of
    each launch move to workgroup groups); the networks whose constant-step
    solve diverges are then solved with the per-pass step (dt_rule 1).  The
    total wall time includes the host round trips and that second solve."""
    import numpy as np

    from paper_2305_07030_amd import dr
    from paper_2305_07030_amd import tune as T
    b = dr.DRBatch(batch, tol=1e-8, max_iter=2_000_000, damping=beta, dt_safety=0.9,
                   tail_at=tail_at, tail_group=tail_group)
    T.apply(b, plans)
    ids = np.arange(len(batch), dtype=np.int32)
    t0 = time.perf_counter()
    b.advance(ids, np.full(len(ids), dr.DR_START_AFFINE, np.int32), 100_000, F=batch.F)
    while True:
        q = b.query(ids)
        run = ids[q["result"] == dr.DR_RUNNING]
        el = time.perf_counter() - t0
        log(f"converge: {el:.1f}s, running {len(run)}, passes max {int(q['iters'].max())}")
        if len(run) == 0 or el > limit_s:
            break
        b.advance(run, np.full(len(run), dr.DR_RESUME, np.int32), 100_000)
    wall1 = time.perf_counter() - t0
    it = q["iters"].copy()
    res = q["result"].copy()
    b.close()
    counts = lambda r: {name: int((r == code).sum()) for name, code in
                        (("converged", dr.DR_CONVERGED), ("max_iter", dr.DR_MAX_ITER),
                         ("nonfinite", dr.DR_NONFINITE), ("running", dr.DR_RUNNING))}
    first = counts(res)
    bad = ids[res == dr.DR_NONFINITE]
    retry = None
    if len(bad):
        t1 = time.perf_counter()
        # with the tail hand-off on, these solves run in workgroup groups too
        # (each group on one XCD; whole rounds of 8 groups must fit on the
        # device's 256 compute units, one 1024-thread workgroup each)
        G = min(16, 256 // (8 * ((len(bad) + 7) // 8))) if tail_at else 0
        G = G if G >= 2 else 0
        rb = dr.DRBatch(batch.subset(bad), tol=1e-8, max_iter=2_000_000, damping=beta, dt_safety=0.9,
                        dt_rule=1, tail_group=G)
        rb.solve()
        r = rb.results()
        rb.close()
        it[bad] = r["iters"]
        res[bad] = r["result"]
        retry = {"networks": bad.tolist(), "workgroups_per_problem": G or 1,
                 "seconds": time.perf_counter() - t1,
                 "passes": r["iters"].tolist(), "result": r["result"].tolist()}
        log(f"converge: per-pass step for {bad.tolist()}: {retry}")
    wall = time.perf_counter() - t0
    return {"wall_s": wall, "constant_step_wall_s": wall1, "updates": float((M * it).sum()),
            "value": float((M * it).sum()) / wall, "unit": "fiber-updates/s",
            "status_counts_constant_step": first, "status_counts": counts(res),
            "per_pass_step_retry": retry, "tail_at": tail_at, "tail_group": tail_group,
            "passes_median": int(np.median(it)), "passes_max": int(it.max()),
            "time_limit_s": limit_s}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="uniform",
                    choices=["uniform", "uniform32", "single", "uneven", "pool", "resident"])
    ap.add_argument("--copies", type=int, default=256, help="resident workload: copies of the network")
    ap.add_argument("--pool-size", type=int, default=4096, help="pool workload: resident networks")
    ap.add_argument("--requests", type=int, default=256, help="pool workload: closed-loop requests")
    ap.add_argument("--state-budget-mib", type=int, default=384,
                    help="pool workload: running-state budget of in-flight solves")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"], help="pool workload")
    ap.add_argument("--rates", default="",
                    help="pool workload: open-loop offered rates as fractions of the closed-loop rate")
    ap.add_argument("--warm", type=int, default=32, help="pool workload: open-loop unmeasured requests")
    ap.add_argument("--measure", type=int, default=256, help="pool workload: open-loop measured requests")
    ap.add_argument("--open-limit", type=float, default=400.0, help="pool workload: seconds per rate")
    ap.add_argument("--passes", type=int, default=20000,
                    help="uneven and resident workloads: passes per network per step")
    ap.add_argument("--no-tune", action="store_true",
                    help="uneven workload: skip the tuner (the library's default plans)")
    ap.add_argument("--converge", action="store_true",
                    help="uneven workload: also solve the batch to convergence")
    ap.add_argument("--converge-limit", type=float, default=900.0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--tail-at", type=int, default=0,
                    help="tail hand-off: problems left running when the rest move to group launches")
    ap.add_argument("--tail-group", type=int, default=0,
                    help="tail hand-off: workgroups per problem (0 = automatic)")
    ap.add_argument("--placement", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-loop", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one plain copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(the sub-problems are independent: a batch splits over GPUs by estimated cost, "
              "with no collective).",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "uneven":
        return uneven_main(args)
    if args.workload == "pool":
        return pool_main(args)
    if args.workload == "resident":
        return resident_main(args)
    # the serving leg's pool is generated in worker processes, before this
    # process touches the GPU
    pool_batch = (make_pool_batch(args.pool_size)
                  if not args.no_serve and args.workload == "uniform" else None)

    import numpy as np
    import torch

    from paper_2305_07030_amd import dr
    from paper_2305_07030_amd import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dr.load()
    prec, stall, bpu = dr.DR_FP64, 0, BYTES_PER_UPDATE
    if args.workload == "uniform":
        batch, beta, tol = I.config_uniform_batch(256), 1e-4, 1e-8
        wl = "256 kNN(k=3) fiber networks, N ~ U{1000..5000}, F = I + sym U(+-0.01), FP64, tol 1e-8"
    elif args.workload == "uniform32":
        # the same batch with FP32 nodal state and force gather (FP64 norms
        # and stress), tol 1e-6, the stall guard on (see fp32_leg)
        batch, beta, tol = I.config_uniform_batch(256), FP32_DAMPING, 1e-6
        prec, stall, bpu = dr.DR_FP32, 50_000, BYTES_PER_UPDATE_FP32
        wl = ("256 kNN(k=3) fiber networks, N ~ U{1000..5000}, F = I + sym U(+-0.01), FP32 state and "
              "gather, FP64 norms and stress, tol 1e-6")
    else:
        batch, beta, tol = I.config_single(), 1e-3, 1e-8
        wl = "1 kNN(k=3) fiber network, N = 500, F = diag(1.01,1,1), FP64, tol 1e-8"
    log("workload:", wl, "networks", len(batch), "fibers", batch.total_fibers)
    copy_calibration(args.copy_mib)
    stream = torch.cuda.current_stream()
    b = dr.DRBatch(batch, tol=tol, damping=beta, dt_safety=0.9, block=args.block,
                   placement=args.placement, tail_at=args.tail_at, tail_group=args.tail_group,
                   precision=prec, stall_window=stall, stream=stream.cuda_stream)
    info = b.info()
    log("launch:", info)
    Fd = torch.tensor(batch.F.reshape(-1, 9), dtype=torch.float64, device="cuda")
    M = np.array([n.n_fibers for n in batch.nets], np.float64)

    for w in range(args.warmup):
        b.solve_device(Fd)
        r = b.results()
        log(f"warmup {w}: passes min/median/max {r['iters'].min()}/{int(np.median(r['iters']))}/{r['iters'].max()}")

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    updates = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        b.solve_device(Fd)
        ev[k][1].record(stream)
        r = b.results()  # waits; sigma, status and pass counts to the host
        updates += float((M * r["iters"]).sum())
        log(f"step {k}: {ev[k][0].elapsed_time(ev[k][1]):.1f} ms kernels")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_s = sum(a.elapsed_time(e) for a, e in ev) / 1e3 / args.steps
    n_conv = int((r["result"] == dr.DR_CONVERGED).sum())
    value = updates / wall
    per_launch = updates / args.steps
    flops = FLOP_PER_UPDATE * per_launch / kern_s
    hbm_equiv = bpu * per_launch / kern_s
    traffic = traffic_for(args.workload)
    ceil = ceilings()
    out = {
        "metric": "fiber-element updates/s (batched persistent launch)",
        "value": value,
        "unit": "fiber-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == dr.DR_FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": wl, "networks": len(batch), "fibers": int(M.sum()),
                   "damping": beta, "dt_safety": 0.9, "block": info["block"],
                   "tail_at": args.tail_at, "tail_group": args.tail_group,
                   "nodes_per_thread": info["nodes_per_thread"], "lds_bytes": info["lds_bytes"],
                   "passes_min": int(r["iters"].min()), "passes_max": int(r["iters"].max()),
                   "passes_median": int(np.median(r["iters"])), "converged": n_conv},
        # achieved = the method's algorithmic bytes (104 B per fiber-update,
        # what the pass would move if the nodal state lived in HBM) per launch
        # over the launch's time; traffic = bytes the launch really moves
        # beyond L2 (rocprofv3 counters), far fewer: the state stays in LDS
        "roofline": {"bound": "hbm", "achieved": hbm_equiv / 1e9, "peak": PEAK_HBM / 1e9,
                     "unit": "GB/s", "frac": hbm_equiv / PEAK_HBM,
                     "traffic": traffic,
                     "achieved_is": f"algorithmic bytes ({bpu:g} B per fiber-update) / launch time",
                     "kernel": ("k_dr_reg" if info["nodes_per_thread"] > 0 else "k_dr_glb") +
                               (" + k_dr_glb group launch (tail hand-off)" if args.tail_at else ""),
                     "kernel_ms": kern_s * 1e3,
                     "bytes_per_update": bpu,
                     "measured_beyond_l2_GBps": traffic / kern_s / 1e9 if traffic else None,
                     "mall_copy_GBps": ceil["mall_copy_GBps"],
                     "hbm_copy_GBps": ceil["hbm_copy_GBps"],
                     "frac_of_mall_copy": hbm_equiv / 1e9 / ceil["mall_copy_GBps"],
                     "fp64_alu_TFLOPs": flops / 1e12,
                     "fp64_alu_frac": flops / PEAK_FP64_VECTOR,
                     "flop_per_update": FLOP_PER_UPDATE},
    }
    if not args.no_loop:
        out["loop_baseline"] = loop_baseline(batch, beta, tol, stream)
        out["loop_baseline"]["speedup_batched_over_loop"] = value / out["loop_baseline"]["value"]
        log("loop baseline:", out["loop_baseline"])
    if not args.no_loop and args.workload == "uniform":
        out["loop_multistream"] = multistream_leg(batch, beta)
        log("loop multistream:", out["loop_multistream"])
    if not args.no_fp32 and args.workload == "uniform":
        out["fp32"] = fp32_leg(batch, stream)
        log("fp32:", {k: v for k, v in out["fp32"].items() if k != "per_network_sigma_rel_err"})
    if not args.no_uneven and args.workload == "uniform":
        out["uneven"] = uneven_leg()
    if not args.no_serve and args.workload == "uniform":
        out["serving"] = serving_leg(pool_batch)
        log("serving:", out["serving"])
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(batch, beta, tol)
        log("cpu baseline:", out["cpu_baseline"])
    b.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
