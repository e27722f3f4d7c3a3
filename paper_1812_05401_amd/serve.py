"""Serving driver: replay a stream of simulation requests through the continuous-batching pool
(or one at a time through the single-simulation API) in real time and measure time-to-result.

Arrival times come with the requests (paper_1812_05401_amd.inputs.serving_requests); a request's
time-to-result runs from its arrival to the moment its final observables are on the host.
"""
import time

import numpy as np

from . import binding as B

# Admission cap for serving: resident lattice nodes enough to fill the GPU four times over
# (256 CUs x 4 resident workgroups x 512 nodes per workgroup x 4).  Measured on the 256-request
# stream at 1.2x capacity: p50 0.21 s / p99 1.00 s with the cap, 0.26 s / 2.04 s without
# (python -m paper_1812_05401_amd.serve --cap-sweep).
DEFAULT_RESIDENT_NODES = 256 * 4 * 512 * 4

# Steps per graph replay of the pool for serving: each replay ends with a host round trip
# (retire, admit) of about 70 us in which the GPU idles.  On the 256-request stream, p50 / p99 at
# 1.2x capacity: 0.21 / 0.65 s with 32 steps, 0.19 / 0.59 s with 64, 0.17 / 0.55 s with 128 and
# 256, 0.18 / 0.56 s with 512 (coarser admission).
SERVING_REPLAY_STEPS = 128


def _percentiles(ttr):
    a = np.asarray(ttr)
    return {"p50_s": float(np.percentile(a, 50)), "p99_s": float(np.percentile(a, 99)),
            "mean_s": float(a.mean()), "max_s": float(a.max())}


def run_pool(requests, budget_bytes, max_slots=128, steps_per_launch=SERVING_REPLAY_STEPS,
             stream=None,
             keep_fields=False, on_result=None, poll_sleep_s=0.0005,
             max_resident_nodes=DEFAULT_RESIDENT_NODES):
    """Replay `requests` through a Pool.  Returns summary statistics (with the number of requests
    that failed: a non-finite or non-positive density) and per-request results."""
    pool = B.Pool(budget_bytes, max_slots=max_slots, steps_per_launch=steps_per_launch,
                  stream=stream)
    if max_resident_nodes:
        pool.set_admission(max_resident_nodes)
    order = sorted(requests, key=lambda r: r.arrival)
    n = len(order)
    t0 = time.perf_counter()
    i = 0
    pending = {}          # pool id -> request
    done_at, results = {}, {}
    max_running = 0
    failed = 0
    while len(done_at) < n:
        now = time.perf_counter() - t0
        while i < n and order[i].arrival <= now:
            rid = pool.submit(order[i].case, order[i].case.steps, keep_fields=keep_fields)
            pending[rid] = order[i]
            i += 1
        running, queued, _ = pool.advance()
        max_running = max(max_running, running)
        t_now = time.perf_counter() - t0
        for rid in list(pending):
            st, _ = pool.status(rid)
            if st in (B.DONE, B.FAILED):
                req = pending.pop(rid)
                res = pool.result(rid, fields=keep_fields)
                failed += st == B.FAILED
                done_at[req.rid] = t_now
                results[req.rid] = res
                if on_result:
                    on_result(req, res)
        if running == 0 and queued == 0 and not pending and i < n:
            wait = order[i].arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.05))
        elif running == 0 and queued == 0 and pending:
            time.sleep(poll_sleep_s)
    wall = time.perf_counter() - t0
    pool.close()
    return _summary(order, done_at, wall, max_running=max_running, failed=failed), results


def run_fifo(requests, stream=None, reduce=True):
    """Baseline: one simulation at a time through the single-simulation API, in arrival order.
    With reduce (the default) each simulation's final mass and body forces come back as the
    pool's results do; the single-simulation API reduces every step for that (the pool only the
    final one), a few percent of its step time, and the summary counts the requests that failed.
    reduce=False skips the reductions and returns no observables."""
    order = sorted(requests, key=lambda r: r.arrival)
    t0 = time.perf_counter()
    done_at = {}
    failed = 0
    for req in order:
        wait = req.arrival - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        sim = B.Simulation(req.case, stream=stream, reduce=reduce)
        sim.step(req.case.steps)
        failed += bool(sim.observables()["status"]) if reduce else 0
        sim.close()
        done_at[req.rid] = time.perf_counter() - t0
    wall = time.perf_counter() - t0
    return _summary(order, done_at, wall, **({"failed": failed} if reduce else {}))


def _summary(order, done_at, wall, **extra):
    ttr = [done_at[r.rid] - r.arrival for r in order]
    lups = sum(r.case.nodes * r.case.steps for r in order)
    first = min(r.arrival for r in order)
    span = max(done_at.values()) - first
    out = {"requests": len(order), "lattice_updates": lups, "makespan_s": span, "wall_s": wall,
           "aggregate_mlups": lups / span / 1e6}
    out.update(_percentiles(ttr))
    out.update(extra)
    return out


def cap_sweep(capacity_glups, loads=(1.2, 0.7), caps=(0, 1_000_000, 2_000_000, 4_000_000),
              n_requests=256, budget_bytes=2 << 30, fifo=False):
    """The serving stream at each offered load (relative to `capacity_glups`) through the pool at
    each admission cap (and, with fifo, one request at a time); one line per run."""
    import dataclasses
    from . import inputs as I
    base = I.serving_requests(n=n_requests, rate_per_s=1.0)
    mean_lups = sum(r.case.nodes * r.case.steps for r in base) / len(base)
    cap_rps = capacity_glups * 1e9 / mean_lups
    for load in loads:
        reqs = [dataclasses.replace(r, arrival=r.arrival / (load * cap_rps)) for r in base]
        for cap in caps:
            st, _ = run_pool(reqs, budget_bytes, max_slots=128, steps_per_launch=SERVING_REPLAY_STEPS,
                             max_resident_nodes=cap)
            print(f"load {load} cap {cap:>8d}: p50 {st['p50_s']:.3f} p99 {st['p99_s']:.3f} "
                  f"mean {st['mean_s']:.3f} max {st['max_s']:.3f} GLUPS {st['aggregate_mlups'] / 1e3:.1f} "
                  f"running<= {st['max_running']} failed {st['failed']}", flush=True)
        if fifo:
            st = run_fifo(reqs)
            print(f"load {load} fifo        : p50 {st['p50_s']:.3f} p99 {st['p99_s']:.3f} "
                  f"mean {st['mean_s']:.3f} max {st['max_s']:.3f} GLUPS {st['aggregate_mlups'] / 1e3:.1f} "
                  f"failed {st['failed']}", flush=True)


def fixed_batch(n, grid, steps, storage="f32", budget_bytes=8 << 30,
                steps_per_launch=SERVING_REPLAY_STEPS, outlet="outflow"):
    """Throughput of a fixed batch: n square requests of one grid (the serving stream's geometry
    draws, all `steps` long, in `storage`, with the zero-gradient outflow or, outlet="convective",
    the convective outlet) submitted at once to a pool without an admission cap,
    timed after the first graph replay (which admits them);
    the same requests through the single-simulation API without reductions, one at a time (each
    finished before the next starts), and all at once, each simulation on a stream of its own.
    A request the pool reports failed (a non-finite or non-positive density) is run alone again
    with reductions, which must fail the same way.  Returns GLUPS of the pool, one at a time and
    the concurrent streams, and the number failed."""
    import torch
    from . import inputs as I
    reqs = I.serving_requests(n=n, nmin=grid, nmax=grid, steps_range=(steps, steps))
    if outlet not in ("outflow", "convective"):
        raise ValueError(f"unknown outlet {outlet!r}")
    for r in reqs:
        r.case.storage = storage
        if outlet == "convective":
            r.case.bc = I.CHANNEL_CONVECTIVE
    lups = sum(r.case.nodes * r.case.steps for r in reqs)
    if steps <= steps_per_launch:
        raise ValueError("the batch must run longer than one graph replay")
    pool = B.Pool(budget_bytes, max_slots=max(n, 1), steps_per_launch=steps_per_launch)
    ids = [pool.submit(r.case, steps) for r in reqs]
    # The first advance admits the batch (allocation, initialisation, mask, graph capture) and
    # runs the first replay; the clock starts when that is done, as the single-simulation legs
    # below start theirs after creating the simulations.
    running, queued, _ = pool.advance()
    if queued:
        raise RuntimeError("the batch does not fit the pool at once")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while True:
        running, queued, _ = pool.advance()
        if running == 0 and queued == 0:
            break
    pool_s = time.perf_counter() - t0
    failed = []
    pool_lups = 0                   # the steps each request ran (a failed one stops early)
    for r, rid in zip(reqs, ids):
        st, done = pool.status(rid)
        pool_lups += r.case.nodes * max(done - steps_per_launch, 0)
        if st == B.FAILED:
            failed.append(r)
        elif st != B.DONE:
            raise RuntimeError(f"request {r.rid} ended in state {st}")
    pool.close()
    sims = [B.Simulation(r.case, stream=None, reduce=False) for r in reqs]   # a stream each
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sim in sims:
        sim.step(steps)
        torch.cuda.synchronize()
    single_s = time.perf_counter() - t0
    for sim in sims:
        sim.close()
    sims = [B.Simulation(r.case, stream=None, reduce=False) for r in reqs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sim in sims:
        sim.step(steps)
    torch.cuda.synchronize()
    streams_s = time.perf_counter() - t0
    for sim in sims:
        sim.close()
    for r in failed:
        sim = B.Simulation(r.case, stream=None, reduce=True)
        sim.step(steps)
        st = sim.observables()["status"]
        sim.close()
        if not st:
            raise RuntimeError(f"request {r.rid} failed in the pool but not alone")
    return pool_lups / pool_s / 1e9, lups / single_s / 1e9, lups / streams_s / 1e9, len(failed)


def main():
    import argparse
    ap = argparse.ArgumentParser(description="serving measurements on one GPU")
    ap.add_argument("--cap-sweep", action="store_true",
                    help="time-to-result of the request stream at each admission cap and load")
    ap.add_argument("--capacity-glups", type=float, default=63.5,
                    help="capacity the offered loads are relative to (the plain FP32 step)")
    ap.add_argument("--loads", default="1.2,0.7")
    ap.add_argument("--caps", default="0,1000000,2000000,4000000")
    ap.add_argument("--fifo", action="store_true", help="also run each load one request at a time")
    ap.add_argument("--batch", default="", metavar="N:GRID:STEPS[:STORAGE[:OUTLET]],...",
                    help="fixed batches through the pool against one at a time, e.g. 24:704:2000 "
                         "or 8:2048:1152:f32:convective")
    args = ap.parse_args()
    if not args.cap_sweep and not args.batch:
        ap.error("nothing to do (try --cap-sweep or --batch)")
    import torch
    torch.cuda.set_device(0)
    B.load()
    for spec in filter(None, args.batch.split(",")):
        f = spec.split(":")
        n, grid, steps = int(f[0]), int(f[1]), int(f[2])
        storage = f[3] if len(f) > 3 else "f32"
        outlet = f[4] if len(f) > 4 else "outflow"
        pool_g, single_g, streams_g, nfail = fixed_batch(n, grid, steps, storage, outlet=outlet)
        print(f"batch {n} x {grid}^2 {storage} {outlet} {steps} steps: pool {pool_g:.1f} GLUPS, "
              f"one at a time {single_g:.1f}, concurrent streams {streams_g:.1f} "
              f"({nfail} failed in both)", flush=True)
    if not args.cap_sweep:
        return
    cap_sweep(args.capacity_glups, tuple(float(x) for x in args.loads.split(",")),
              tuple(int(x) for x in args.caps.split(",")), fifo=args.fifo)


if __name__ == "__main__":
    main()
