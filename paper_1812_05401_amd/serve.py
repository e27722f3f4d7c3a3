"""Serving driver: replay a stream of simulation requests through the continuous-batching pool
(or one at a time through the single-simulation API) in real time and measure time-to-result.

Arrival times come with the requests (paper_1812_05401_amd.inputs.serving_requests); a request's
time-to-result runs from its arrival to the moment its final observables are on the host.
"""
import time

import numpy as np

from . import binding as B

# Admission cap for serving: resident lattice nodes enough to fill the GPU four times over
# (256 CUs x 8 resident workgroups x 256 nodes per workgroup x 4).  Measured on the 256-request
# stream at 1.2x capacity: p50 0.20 s / p99 1.07 s with the cap, 0.29 s / 2.50 s without.
DEFAULT_RESIDENT_NODES = 256 * 8 * 256 * 4


def _percentiles(ttr):
    a = np.asarray(ttr)
    return {"p50_s": float(np.percentile(a, 50)), "p99_s": float(np.percentile(a, 99)),
            "mean_s": float(a.mean()), "max_s": float(a.max())}


def run_pool(requests, budget_bytes, max_slots=128, steps_per_launch=64, stream=None,
             keep_fields=False, on_result=None, poll_sleep_s=0.0005,
             max_resident_nodes=DEFAULT_RESIDENT_NODES):
    """Replay `requests` through a Pool.  Returns summary statistics and per-request results."""
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
    return _summary(order, done_at, wall, max_running=max_running), results


def run_fifo(requests, stream=None):
    """Baseline: one simulation at a time through the single-simulation API, in arrival order."""
    order = sorted(requests, key=lambda r: r.arrival)
    t0 = time.perf_counter()
    done_at = {}
    for req in order:
        wait = req.arrival - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        sim = B.Simulation(req.case, stream=stream, reduce=False)
        sim.step(req.case.steps)
        sim.observables()
        sim.close()
        done_at[req.rid] = time.perf_counter() - t0
    wall = time.perf_counter() - t0
    return _summary(order, done_at, wall)


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
