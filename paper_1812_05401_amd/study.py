"""Long runs with per-step observables: the force series of a simulation (drained from the
device ring in chunks) plus density/velocity snapshots, and the comparison of storage formats
against the FP64 run of the same case (velocity L2 of Eq. 20, C_D / C_L / St of Eqs. 22-23)."""
import copy
import time

import numpy as np

from . import analysis as A
from . import binding as B


def run_series(case, steps, storage=None, snapshots=(), chunk=4000, stream=None, me_every=0,
               log=None):
    """Run `case` for `steps` steps.  Returns the per-step mass and body-0 force series, the
    fields at the requested snapshot steps, the mask and the wall time; with me_every > 0 also
    the body-0 momentum-exchange force sampled every me_every steps.  `log` receives a progress
    line about every twentieth of the run."""
    c = copy.copy(case)
    if storage:
        c.storage = storage
    sim = B.Simulation(c, stream=stream, ring=chunk + 8)
    mass = np.empty(steps)
    fx = np.empty(steps)
    fy = np.empty(steps)
    snaps = {}
    marks = sorted(set(s for s in snapshots if 0 < s <= steps))
    if me_every:
        chunk = min(chunk, me_every)
    me = []
    done = 0
    every = max(steps // 20, 1)
    t0 = time.perf_counter()
    while done < steps:
        n = min(chunk, steps - done)
        nxt = [m for m in marks if m > done]
        if nxt:
            n = min(n, nxt[0] - done)
        sim.step(n)
        ser = sim.force_series(done, n)
        mass[done:done + n] = ser[:, 0]
        fx[done:done + n] = ser[:, 1]
        fy[done:done + n] = ser[:, 2]
        if log and (done + n) // every > done // every:
            log(f"{c.name}/{c.storage}: step {done + n} of {steps}, "
                f"{time.perf_counter() - t0:.1f} s")
        done += n
        if done in marks:
            snaps[done] = sim.fields()
        if me_every and done % me_every == 0:
            mfx, mfy = sim.momentum_exchange()
            me.append((done - 1, mfx[0], mfy[0]))
    obs = sim.observables()
    wall = time.perf_counter() - t0
    mask = sim.mask()
    sim.close()
    return {"mass": mass, "fx": fx, "fy": fy, "snapshots": snaps, "mask": mask,
            "status": obs["status"], "wall_s": wall, "storage": c.storage,
            "momentum_exchange": np.array(me).reshape(-1, 3)}


def compare_storages(case, steps, storages=("f64", "f32", "f32d", "f16s", "f16sr", "bf16s", "bf16sr"), snapshots=(1000, 10000),
                     stats_from=None, stream=None, log=None, dump=None, me_every=0):
    """Run `case` in every storage format and compare each with the FP64 run (and with FP32).
    `dump`: optional .npz path for the raw per-step series."""
    stats_from = steps // 2 if stats_from is None else stats_from
    runs = {}
    for st in storages:
        runs[st] = run_series(case, steps, st, snapshots, stream=stream, me_every=me_every, log=log)
        if log:
            log(f"{case.name}/{st}: {steps} steps in {runs[st]['wall_s']:.1f} s, status {runs[st]['status']}")
    if dump:
        np.savez_compressed(dump, **{f"{st}_{k}": r[k] for st, r in runs.items()
                                     for k in ("mass", "fx", "fy", "momentum_exchange")})
    u, d = case.u_in[0], case.diameter
    out = {"workload": case.name, "steps": steps, "stats_from_step": stats_from, "storages": {}}
    ref = runs.get("f64")
    for st, r in runs.items():
        ent = {"status": int(r["status"]), "wall_s": round(r["wall_s"], 2),
               "mass_drift": float((r["mass"][-1] - r["mass"][0]) / r["mass"][0])}
        ent.update(A.wake_statistics(r["fx"], r["fy"], u, d, first=stats_from))
        me = r["momentum_exchange"]
        if len(me):
            sel = me[:, 0] >= stats_from
            cd_me, cl_me = A.force_coefficients(me[sel, 1], me[sel, 2], u, d)
            ent["C_Dave_momentum_exchange"] = float(cd_me.mean())
            ent["C_Lrms_momentum_exchange"] = float(np.sqrt(np.mean((cl_me - cl_me.mean()) ** 2)))
            ent["momentum_exchange_samples"] = int(sel.sum())
        fluid = r["mask"] == 0
        for base_name in ("f64", "f32"):
            base = runs.get(base_name)
            if base is None or base_name == st:
                continue
            for s, (rho, ux, uy) in r["snapshots"].items():
                _, bux, buy = base["snapshots"][s]
                ent[f"velocity_l2_vs_{base_name}_step{s}"] = A.l2_error(np.stack([ux, uy]), np.stack([bux, buy]), fluid)
            bs = A.wake_statistics(base["fx"], base["fy"], u, d, first=stats_from)
            for k in ("C_Dave", "C_Lrms", "St", "St_spectral"):
                if ent[k] is not None and bs[k]:
                    ent[f"{k}_rel_diff_vs_{base_name}"] = (ent[k] - bs[k]) / abs(bs[k])
        out["storages"][st] = ent
    return out
