"""Benchmark of the fused VP-LBM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

A "step" is one lattice update of the whole grid: pull-streaming, edge rules, mask fetch,
moments, penalization, collision, store, and the FP64 mass/force reductions.  The default
workload is the 8192 x 2048 transversely oscillating cylinder (VP-MRT, FP32 storage, Zou-He
inlet, outflow, free-slip walls, disk D = 96, Re = 300, mask and solid velocity rebuilt on the
device every step).  Its two population buffers (1.2 GB) far exceed the 256 MB Infinity Cache, so
the step streams from HBM and the line's `roofline` is an HBM figure.  The library runs three
steps per launch (the intermediate steps kept in LDS); `two_steps_per_launch` and
`one_step_per_launch` time the same workload with two steps per launch and with one, the
memory-bound kernel.  Beside it the line carries `cache_resident` (the
2048 x 512 cylinder wake, whose 75 MB of buffers fit in the cache: MLUPS only),
`taylor_couette_128` (the 128 x 128 FP64 case, launch-bound: MLUPS only), `reduced_precision`
(the 8192 x 2048 cylinder in every storage format), `paper_cylinder_re500` (the paper's
6048 x 2016 Re = 500 case with its convective outlet), a square FP32 sweep, the measured copy
ceiling, the serving workload and the FP64 oracle on the host's cores (`cpu_baseline`).

Prints one JSON line.  Inputs are synthetic (seeded geometry, uniform start) and resident on the
GPU before timing starts.  `--copy-probe BYTES` instead times a plain device copy (the measured
HBM ceiling and the calibration kernel for the FETCH_SIZE/WRITE_SIZE counters).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM roofline (D2Q9 VP-MRT step); served p50/p99 time-to-result"
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E datasheet peak
# FP32 FMA issue rate without packed FP32 (which the build disables): 256 CUs x 4 SIMDs x 16 lanes
# x 2.4 GHz lane-instructions per second (the datasheet's 157.3 TFLOP/s halved for packing and
# halved again for counting an FMA as two flops).  Independent FMA chains reach 35.6 T/s of it;
# some other instruction mixes issue faster, so a kernel's VALU rate against it is a diagnostic.
VALU_FMA_RATE_T = 256 * 4 * 16 * 2.4e9 / 1e12


from paper_1812_05401_amd.counters import source_digest  # noqa: E402  (the counter tables carry it)


def pattern_ceilings(nx, ny, launches=64):
    """The step kernels' access patterns with a trivial per-node update (libvplbm_probes.so) on an
    nx x ny FP32 lattice: microseconds per launch with 1, 2 and 3 updates per launch (the one-step
    kernel's 128 x 2 workgroups, the two-step kernel's 128 x 8 tiles, the three-step kernel's
    64 x 14 tiles), the best of three timings.  A probe needs the lattice to be a whole number of tiles: otherwise it
    runs on the largest such lattice inside and its time is scaled by the node count.  The FP32 FMA issue rate of
    independent chains comes with it."""
    from paper_1812_05401_amd import probes as P
    out = {"lattice": f"{nx}x{ny}", "storage": "f32", "bytes_per_node_per_launch": 73}
    for spl, tile in ((1, (128, 2)), (2, (128, 8)), (3, (64, 14))):
        nxt, nyt = nx - nx % tile[0], ny - ny % tile[1]
        us = min(P.pattern_us(nxt, nyt, spl, tile, launches) for _ in range(3)) * (nx * ny) / (nxt * nyt)
        out[f"steps_per_launch_{spl}"] = {"tile": list(tile), "us_per_launch": round(us, 2),
                                          "us_per_step": round(us / spl, 2),
                                          "gbs": round(73 * nx * ny / (us * 1e-6) / 1e9, 1)}
    out["fma_lane_per_s_t"] = round(P.fma_rate(20) / 1e12, 3)
    return out


def cache_resident(case):
    """Whether the two population buffers fit in the 256 MB Infinity Cache."""
    eb = {"f64": 8, "f32": 4, "f32d": 4}.get(case.storage, 2)
    return case.nx * case.ny * 2 * 9 * eb < 256e6


def profile_entry(table, workload, storage, steps_per_launch):
    """An entry of a committed counter summary (profiles/<table>.json) for this workload and
    kernel, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{table}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        tab = json.load(f)
    ent = tab.get(f"{workload}/{storage}/{steps_per_launch}")
    if not ent or ent.get("source_digest") != source_digest():
        return None
    return ent


def measured_traffic(workload, storage, steps_per_launch=1):
    """HBM bytes per step-kernel launch from the committed FETCH_SIZE/WRITE_SIZE summary."""
    ent = profile_entry("traffic", workload, storage, steps_per_launch)
    return ent and ent.get("bytes_per_launch")


def time_workload(case, steps, warmup, storage=None, spl=3):
    """Time `steps` steps of `case` after `warmup`, with at most `spl` steps per launch: 1 creates
    the simulation with VPLBM_TWO_STEP=0, 2 with VPLBM_THREE_STEP=0; the library takes as many as
    the case allows (three for binary32 storage, else two)."""
    import torch
    from paper_1812_05401_amd import binding as B
    if storage:
        case.storage = storage
    # A non-default torch stream: its handle is what the library orders its work on and what
    # the timing events are recorded on (the default stream's handle is NULL, which the C ABI
    # reads as "use a stream of your own").
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    want = {"VPLBM_TWO_STEP": "1" if spl >= 2 else "0", "VPLBM_THREE_STEP": "1" if spl >= 3 else "0"}
    old = {k: os.environ.get(k) for k in want}
    os.environ.update(want)
    try:
        sim = B.Simulation(case, stream=int(stream.cuda_stream))
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k)
            else:
                os.environ[k] = v
    assert sim.stream == stream.cuda_stream
    spl = sim.steps_per_launch
    sim.step(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    sim.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    obs = sim.observables()
    sim.close()
    if obs["status"] != 0:
        raise RuntimeError(f"{case.name}: unstable")
    bpu = B.vplbm_bytes_per_update(case.storage)
    # One launch updates every node spl times (the graph's step-counter kernel, one per 128 steps,
    # and, with moving bodies, the kernel that rebuilds their masks before each launch are included
    # in the launch time).  The bytes it moves are one read and one write of the planes plus the
    # mask whatever spl is: the multi-step kernels keep the intermediate steps on chip.
    launch_s = gpu_ms / 1e3 / steps * spl
    # moving bodies: a launch of several steps reads the mask of each of its steps (1 B per node
    # and step more)
    moving = any(b["freq"] != 0 and (b["ax"] != 0 or b["ay"] != 0) for b in case.bodies)
    bytes_launch = (bpu + (spl - 1 if moving else 0)) * case.nodes
    hbm = bytes_launch / launch_s / 1e9
    # The per-update figure: bpu bytes (9 loads, 9 stores, the mask) for each of the spl lattice
    # updates of a launch, over the same launch time.  Above 1 for the multi-step kernels, which
    # move those bytes once per spl updates.
    per_update = bpu * spl * case.nodes / launch_s / 1e9
    kernel = {1: "vplbm::step_kernel", 2: "vplbm::step2_kernel", 3: "vplbm::step3_kernel"}[spl]
    roof = {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(hbm / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(case.name, case.storage, spl),
            "frac_per_update_bytes": round(per_update / HBM_PEAK_GBS, 4),
            "achieved_per_update_bytes": round(per_update, 1),
            "bytes_per_update": bpu,
            "kernel": kernel, "lattice_updates_per_launch": spl, "launch_us": round(launch_s * 1e6, 3),
            "bytes_per_launch": bytes_launch, "bytes_per_node_per_launch": bytes_launch // case.nodes}
    valu = profile_entry("valu", case.name, case.storage, spl)
    if valu:
        # The kernel's VALU instructions (SQ_INSTS_VALU x 64 lanes per launch, from the committed
        # counter summary) over the same launch time: how busy the vector ALUs are beside HBM.
        t = valu["valu_lane_instr_per_launch"] / launch_s / 1e12
        roof["valu"] = {"achieved": round(t, 3), "fma_issue_rate": round(VALU_FMA_RATE_T, 3),
                        "unit": "T lane-instructions/s", "ratio": round(t / VALU_FMA_RATE_T, 4),
                        "per_lattice_update": valu["valu_per_lattice_update"]}
    return {
        "workload": case.name, "nx": case.nx, "ny": case.ny, "storage": case.storage,
        "collision": case.collision, "steps": steps, "steps_per_launch": spl,
        "mlups": case.nodes * steps / (gpu_ms / 1e3) / 1e6,
        "ms_per_step": gpu_ms / steps, "wall_s": wall, "mass": obs["mass"],
        # what one step per launch would have to move at this rate (not a measured bandwidth)
        "one_step_equivalent_gbs": round(bpu * case.nodes * steps / (gpu_ms / 1e3) / 1e9, 1),
        "roofline": roof,
    }


def host_threads():
    """Threads the oracle may use: the processors this process may run on, at most the
    OMP_NUM_THREADS the environment sets (the share of the host's CPUs a job is given)."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(n, 1)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_mlups(case, steps, threads):
    """The FP64 oracle (test infrastructure, not the product path) on `steps` steps of `case`:
    MLUPS over the step loop alone, every node counted."""
    import oracle as O
    kinds = {"disk": O.DISK, "rect": O.RECT, "disk_outside": O.DISK_OUTSIDE}
    bcs = {"periodic": O.PERIODIC, "velocity": O.VELOCITY, "outflow": O.OUTFLOW,
           "freeslip": O.FREESLIP, "convective": O.CONVECTIVE}
    s = O.OracleSim(case.nx, case.ny, O.MRT if case.collision == "mrt" else O.SRT, tau=case.tau,
                    lam=case.lam, eta=case.eta, bc=tuple(bcs[b] for b in case.bc), u_in=case.u_in,
                    threads=threads)
    s.set_bodies([O.make_body(kinds[b["kind"]], b["cx"], b["cy"], b["r"], b["hx"], b["hy"],
                              b["ux"], b["uy"], b["omega"], b["ax"], b["ay"], b["freq"])
                  for b in case.bodies])
    s.init_uniform(case.rho0, *case.u0)
    t0 = time.perf_counter()
    s.step(steps)
    dt = time.perf_counter() - t0
    used = s.threads
    s.close()
    return {"workload": case.name, "nodes": case.nodes, "collision": case.collision,
            "steps": steps, "threads": used, "seconds": round(dt, 3),
            "mlups": round(case.nodes * steps / dt / 1e6, 3)}


def cpu_baseline(head, samples):
    """The FP64 oracle timed on the host: one thread and every thread this process may use, on a
    bounded sample of the headline workload and of the other workloads in `samples` [(case,
    steps_one_thread, steps_all_threads)].  The thread count does not change the oracle's
    results (its per-step sums are serial)."""
    nthr = host_threads()
    legs = []
    for case, s1, sn in samples:
        for th, n in ((1, s1), (nthr, sn)):
            r = oracle_mlups(case, n, th)
            legs.append(r)
            print(f"# cpu oracle {case.name}: {r['threads']} thread(s), {n} steps, "
                  f"{r['mlups']:.2f} MLUPS", file=sys.stderr, flush=True)
    main = [r for r in legs if r["workload"] == head.name]
    one = next(r for r in main if r["threads"] == 1)
    allc = next(r for r in main if r["threads"] != 1) if nthr > 1 else one
    return {"value": allc["mlups"], "unit": "MLUPS", "cores": allc["threads"], "kind": "oracle",
            "sample": f"{allc['steps']} steps of {head.name} ({head.nodes} nodes), FP64 oracle, "
                      f"{head.collision.upper()} in moment space, {allc['threads']} threads, "
                      f"{allc['seconds']:.1f} s; one thread: {one['steps']} steps, "
                      f"{one['mlups']:.2f} MLUPS",
            "threads_1": one, "threads_all": allc, "nproc": os.cpu_count(),
            "threads_available": nthr, "cpu_model": cpu_model(), "legs": legs}


def serving_leg(n_requests, loads, budget_bytes, fifo_loads):
    """The serving workload: Poisson arrivals of VP-MRT FP32 channel simulations replayed in real
    time through the continuous-batching pool at offered loads relative to the measured capacity
    of the plain FP32 step, beside a one-at-a-time FIFO baseline on the same GPU."""
    import dataclasses
    from paper_1812_05401_amd import inputs as I
    from paper_1812_05401_amd import serve
    base = I.serving_requests(n=n_requests, rate_per_s=1.0)
    mean_lups = sum(r.case.nodes * r.case.steps for r in base) / len(base)
    # capacity of the plain FP32 step on a grid of the mean size of the stream
    nmean = int(round((sum(r.case.nodes for r in base) / len(base)) ** 0.5 / 32)) * 32
    probe = I.cylinder_wake(nmean, nmean, d=nmean / 8, x0=nmean / 4, re=200.0, steps=2000)
    cap = time_workload(probe, 2000, 200)
    cap_rps = cap["mlups"] * 1e6 / mean_lups
    out = {"workload": f"serving_{n_requests}_poisson", "requests": n_requests,
           "mean_lattice_updates_per_request": mean_lups, "budget_bytes": budget_bytes,
           "plain_fp32_step": {"grid": f"{nmean}x{nmean}", "mlups": round(cap["mlups"], 1)},
           "capacity_requests_per_s": cap_rps, "runs": {}}

    def at_load(load):
        rate = load * cap_rps
        return [dataclasses.replace(r, arrival=r.arrival / rate) for r in base]

    out["max_resident_nodes"] = serve.DEFAULT_RESIDENT_NODES
    out["steps_per_replay"] = serve.SERVING_REPLAY_STEPS
    for load in loads:
        stats, _ = serve.run_pool(at_load(load), budget_bytes, max_slots=128,
                                  steps_per_launch=serve.SERVING_REPLAY_STEPS)
        out["runs"][f"pool_load_{load}"] = stats
        print(f"# serving pool load {load}: p50 {stats['p50_s']:.2f} s p99 {stats['p99_s']:.2f} s "
              f"{stats['aggregate_mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    # the same pool without the admission cap, at the highest load
    stats, _ = serve.run_pool(at_load(max(loads)), budget_bytes, max_slots=128,
                              steps_per_launch=serve.SERVING_REPLAY_STEPS,
                              max_resident_nodes=0)
    out["runs"][f"pool_uncapped_load_{max(loads)}"] = stats
    print(f"# serving pool (no admission cap) load {max(loads)}: p50 {stats['p50_s']:.2f} s "
          f"p99 {stats['p99_s']:.2f} s", file=sys.stderr, flush=True)
    for load in fifo_loads:
        stats = serve.run_fifo(at_load(load))
        out["runs"][f"fifo_load_{load}"] = stats
        print(f"# serving fifo load {load}: p50 {stats['p50_s']:.2f} s p99 {stats['p99_s']:.2f} s "
              f"{stats['aggregate_mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    return out


def measure_copy(nbytes, reps):
    """Device-to-device copy of `nbytes` (torch), read + write bandwidth: the measured ceiling a
    streaming kernel is compared with beside the datasheet peak."""
    import torch
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_blit = timed(lambda: b.copy_(a))                      # the runtime's copy (blit kernel)
    ms_ew = timed(lambda: torch.mul(a, 1.0, out=b))          # an elementwise kernel
    del a, b
    gbs = lambda ms: round(2 * 4 * n / (ms / 1e3) / 1e9, 1)
    return {"copy_bytes": 4 * n, "reps": reps, "ms_blit": ms_blit, "ms_elementwise": ms_ew,
            "gbs_blit": gbs(ms_blit), "gbs_elementwise": gbs(ms_ew),
            "gbs_read_plus_write": max(gbs(ms_blit), gbs(ms_ew))}


def copy_probe(nbytes, reps):
    print(json.dumps(measure_copy(nbytes, reps)), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1024)     # 8 graph replays of 128 steps
    ap.add_argument("--warmup", type=int, default=128)
    ap.add_argument("--workload", default="oscillating_cylinder_8192x2048")
    ap.add_argument("--storage", default="", help="storage format of the workload (default: its own)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the objects beside the headline")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES")
    ap.add_argument("--probes", action="store_true",
                    help="instead of the benchmark: the access-pattern ceilings (trivial per-node "
                         "update) of the benchmark lattices and the FMA issue rate, one JSON line")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving workload")
    ap.add_argument("--precision-study", default="", metavar="WORKLOAD",
                    help="instead of the benchmark: run WORKLOAD (cylinder_wake_2048x512, "
                         "cylinder_wake_8192x2048, paper_cylinder_re500 or "
                         "oscillating_cylinder_8192x2048) in the storage formats of --storages for "
                         "--steps steps and print the comparison against FP64")
    ap.add_argument("--dump", default="", help="with --precision-study: .npz for the series")
    ap.add_argument("--sweep", default="", choices=["", "fig3", "fig12", "fig12_readings", "table1",
                                                    "fig5", "fig14"],
                    help="instead of the benchmark: run one of the paper's parameter sweeps "
                         "through the serving pool and print the L2 errors (fig5, fig14: steps "
                         "to convergence under the early stop)")
    ap.add_argument("--stop", type=float, default=0.0,
                    help="with --sweep: retire each point early once its convergence residual "
                         "over --stop-every steps is below this tolerance")
    ap.add_argument("--stop-every", type=int, default=1000)
    ap.add_argument("--sweep-steps-scale", type=int, default=1,
                    help="with --sweep fig12_readings: run each point this many times longer")
    ap.add_argument("--me-every", type=int, default=0,
                    help="with --precision-study: sample the momentum-exchange force every N steps")
    ap.add_argument("--storages", default="f64,f32,f32d,f16s,f16sr,bf16s,bf16sr",
                    help="with --precision-study: storage formats to run")
    ap.add_argument("--stats-from", type=int, default=-1,
                    help="with --precision-study: first step of the statistics window (default: half)")
    ap.add_argument("--serving-requests", type=int, default=256)
    ap.add_argument("--force-regions", default="", metavar="WORKLOAD",
                    help="instead of the benchmark: split the drag of WORKLOAD (cylinder_wake_2048x512 "
                         "or cylinder_wake_8192x2048) into the body's surface layer and interior, "
                         "for the storages of --storages (time means from --stats-from on)")
    ap.add_argument("--sensitivity", default="", choices=["", "re500"],
                    help="instead of the benchmark: run the variants of the paper's Re = 500 "
                         "cylinder (outlet rule, eta, inlet and outlet distance, collision, "
                         "resolution, channel height) and print C_D, C_Lrms and St of each")
    ap.add_argument("--variants", default="",
                    help="with --sensitivity: comma-separated labels of the variants to run (all)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: there is no multi-GPU path (asked for "
              f"--gpus {args.gpus}).  Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe(args.copy_probe, max(args.steps, 1))
        return
    if args.probes:
        res = {"probes": [pattern_ceilings(nx, ny) for nx, ny in ((8192, 2048), (2048, 512), (6048, 2016))]}
        print(json.dumps(res), flush=True)
        return

    from paper_1812_05401_amd import binding as B
    from paper_1812_05401_amd import inputs as I
    B.load()
    if args.sweep:
        from paper_1812_05401_amd import sweeps
        pts = {"fig3": sweeps.fig3_shear, "fig12": sweeps.fig12_couette,
               "fig12_readings": lambda: sweeps.fig12_readings(args.sweep_steps_scale),
               "table1": sweeps.table1_grids, "fig5": sweeps.fig5_convergence,
               "fig14": sweeps.fig14_convergence}[args.sweep]()
        stop = (args.stop, args.stop_every) if args.stop > 0 else sweeps.CONVERGENCE_STOP.get(args.sweep)
        t0 = time.perf_counter()
        res = sweeps.run(pts, stop=stop)
        wall = time.perf_counter() - t0
        lups = sum(p.case.nodes * r["steps"] for p, r in zip(pts, res))
        print(json.dumps({"sweep": args.sweep, "points": len(pts), "stop": stop,
                          "lattice_updates": lups, "wall_s": wall, "mlups": lups / wall / 1e6,
                          "results": res}), flush=True)
        return
    if args.force_regions:
        from paper_1812_05401_amd import study
        mk = {"cylinder_wake_2048x512": I.cylinder_wake_2048x512,
              "cylinder_wake_8192x2048": lambda: I.cylinder_wake_8192x2048("f32")}[args.force_regions]
        res = study.force_region_study(mk(), storages=tuple(args.storages.split(",")),
                                       steps=args.steps,
                                       first=args.steps // 2 if args.stats_from < 0 else args.stats_from,
                                       log=lambda m: print("# " + m, file=sys.stderr, flush=True))
        print(json.dumps(res), flush=True)
        return
    if args.sensitivity:
        from paper_1812_05401_amd import study
        cases = I.paper_cylinder_sensitivity(args.storage or "f32")
        if args.variants:
            keep = args.variants.split(",")
            cases = [c for c in cases if c.name.replace("paper_cylinder_re500_", "") in keep]
        res = study.sensitivity(cases, dump_dir=os.path.dirname(args.dump) if args.dump else None,
                                log=lambda m: print("# " + m, file=sys.stderr, flush=True))
        print(json.dumps({"sensitivity": args.sensitivity, "runs": res}), flush=True)
        return
    if args.precision_study:
        from paper_1812_05401_amd import study
        mk = {"cylinder_wake_2048x512": I.cylinder_wake_2048x512,
              "cylinder_wake_8192x2048": lambda: I.cylinder_wake_8192x2048("f32"),
              "paper_cylinder_re500": I.paper_cylinder_re500,
              "oscillating_cylinder_8192x2048": I.oscillating_cylinder_8192x2048}[args.precision_study]
        res = study.compare_storages(mk(), args.steps, dump=args.dump or None,
                                     storages=tuple(args.storages.split(",")),
                                     me_every=args.me_every,
                                     stats_from=None if args.stats_from < 0 else args.stats_from,
                                     log=lambda m: print("# " + m, file=sys.stderr, flush=True))
        print(json.dumps(res), flush=True)
        return
    workloads = {
        "cylinder_wake_2048x512": I.cylinder_wake_2048x512,
        "taylor_couette_128": I.taylor_couette_128,
        "oscillating_cylinder_8192x2048": I.oscillating_cylinder_8192x2048,
        "cylinder_wake_8192x2048": lambda: I.cylinder_wake_8192x2048("f32"),
    }
    case = workloads[args.workload]()
    if args.storage:
        case.storage = args.storage
    main_res = time_workload(case, args.steps, args.warmup)
    print(f"# {case.name}: {main_res['mlups']:.0f} MLUPS, {main_res['ms_per_step'] * 1e3:.2f} us/step",
          file=sys.stderr, flush=True)

    line = {
        "metric": METRIC, "value": round(main_res["mlups"], 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 6), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "f32d": "f64", "f16s": "f32", "bf16s": "f32", "f16sr": "f32", "bf16sr": "f32"}[case.storage],
        "data": "synthetic",
        "config": {"workload": case.name, "nx": case.nx, "ny": case.ny,
                   "collision": case.collision, "storage": case.storage, "tau": case.tau,
                   "lambda": case.lam, "eta": case.eta, "bc": list(case.bc),
                   "bodies": len(case.bodies),
                   "moving_bodies": any(b["freq"] != 0 for b in case.bodies),
                   "reductions": "fp64 mass + body force, every step",
                   "cache_resident": cache_resident(case)},
        "roofline": main_res["roofline"],
        "steps_per_launch": main_res["steps_per_launch"],
        "one_step_equivalent_gbs": main_res["one_step_equivalent_gbs"],
    }
    if not args.no_extra:
        # the same access pattern with a trivial update: the ceiling of the pattern itself
        pc = pattern_ceilings(case.nx, case.ny)
        line["pattern_ceilings"] = pc
        ceil = pc.get(f"steps_per_launch_{main_res['steps_per_launch']}")
        if ceil:
            line["roofline"]["pattern_ceiling_us"] = ceil["us_per_launch"]
            line["roofline"]["frac_of_pattern_ceiling"] = round(
                ceil["us_per_launch"] / line["roofline"]["launch_us"], 4)
    if main_res["steps_per_launch"] >= 2:
        # the same workload with fewer steps per launch: one (the memory-bound kernel and its
        # roofline) and, under three, two
        for spl, key in ((2, "two_steps_per_launch"), (1, "one_step_per_launch")):
            if spl >= main_res["steps_per_launch"]:
                continue
            r = time_workload(workloads[args.workload](), args.steps, args.warmup,
                              storage=args.storage or None, spl=spl)
            line[key] = {k: r[k] for k in ("mlups", "ms_per_step", "roofline")}
            c = pc.get(f"steps_per_launch_{spl}") if not args.no_extra else None
            if c:
                line[key]["roofline"]["pattern_ceiling_us"] = c["us_per_launch"]
                line[key]["roofline"]["frac_of_pattern_ceiling"] = round(
                    c["us_per_launch"] / line[key]["roofline"]["launch_us"], 4)
            print(f"# {case.name} {spl} step(s) per launch: {r['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    if not args.no_extra:
        # the 2048 x 512 wake: buffers inside the Infinity Cache, so MLUPS only
        c2 = I.cylinder_wake_2048x512()
        r = time_workload(c2, 6144, 768)
        line["cache_resident"] = {"workload": c2.name, "storage": c2.storage, "steps": 6144,
                                  "mlups": round(r["mlups"], 1), "ms_per_step": r["ms_per_step"],
                                  "steps_per_launch": r["steps_per_launch"],
                                  "note": "75 MB of buffers inside the 256 MB Infinity Cache: MLUPS only"}
        print(f"# {c2.name}: {r['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        # the 128 x 128 FP64 Taylor-Couette case over its 5000 steps: launch-bound, MLUPS only
        c1 = I.taylor_couette_128()
        r = time_workload(c1, 5000, 200)
        line["taylor_couette_128"] = {"workload": c1.name, "storage": c1.storage, "steps": 5000,
                                      "mlups": round(r["mlups"], 1), "ms_per_step": r["ms_per_step"],
                                      "steps_per_launch": r["steps_per_launch"],
                                      "note": "16,384 nodes: launch-bound, MLUPS only"}
        print(f"# {c1.name}: {r['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        red = {}
        for st in ("f64", "f32", "f32d", "f16s", "f16sr", "bf16s", "bf16sr"):
            c = I.cylinder_wake_8192x2048(st)
            r = time_workload(c, 400, 40)
            red[st] = {k: r[k] for k in ("mlups", "ms_per_step", "steps_per_launch", "roofline")}
            print(f"# {c.name}/{st}: {r['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        line["reduced_precision"] = {"workload": "cylinder_wake_8192x2048", **red}
        # the paper's own Re = 500 cylinder (6048 x 2016, SRT, convective outlet), FP32
        pcr = {}
        for spl, key in ((3, "three_steps_per_launch"), (2, "two_steps_per_launch"),
                         (1, "one_step_per_launch")):
            r = time_workload(I.paper_cylinder_re500("f32"), 402, 42, spl=spl)
            pcr[key] = {k: r[k] for k in ("mlups", "ms_per_step", "steps_per_launch", "roofline")}
            print(f"# paper_cylinder_re500 ({spl} per launch): {r['mlups']:.0f} MLUPS",
                  file=sys.stderr, flush=True)
        line["paper_cylinder_re500"] = {"workload": "paper_cylinder_re500", "storage": "f32", **pcr}
        # FP32 square channels from cache-resident to far beyond the 256 MB Infinity Cache
        sweep = []
        for n, steps in ((2048, 400), (4096, 200), (8192, 60)):
            c = I.cylinder_wake(n, n, d=n / 8, x0=n / 4, re=200.0, steps=steps)
            r = time_workload(c, steps, 20)
            sweep.append({"grid": f"{n}x{n}", "buffers_bytes": 2 * 9 * 4 * n * n,
                          "mlups": round(r["mlups"], 1), "ms_per_step": r["ms_per_step"],
                          "steps_per_launch": r["steps_per_launch"],
                          "one_step_equivalent_gbs": r["one_step_equivalent_gbs"]})
            print(f"# square {n}x{n}: {r['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        line["square_sweep_f32"] = sweep
        cp = measure_copy(1 << 30, 20)
        line["copy_probe"] = cp
        for obj in [line["roofline"], line.get("one_step_per_launch", {}).get("roofline")]:
            if not obj:
                continue
            obj["frac_of_copy"] = round(obj["achieved"] / cp["gbs_read_plus_write"], 4)
    if not args.no_serving:
        line["serving"] = serving_leg(args.serving_requests, (0.7, 1.2), 2 << 30, (0.7, 1.2))
    if not args.no_cpu_baseline:
        # bounded samples (about 20 s of oracle work on a 16-thread share): the headline workload,
        # the 2048 x 512 wake and the whole 5000-step 128 x 128 Taylor-Couette run
        line["cpu_baseline"] = cpu_baseline(case, [(workloads[args.workload](), 2, 12),
                                                   (I.cylinder_wake_2048x512(), 30, 300),
                                                   (I.taylor_couette_128(), 5000, 5000)])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
