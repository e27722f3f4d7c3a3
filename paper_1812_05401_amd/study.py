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


def sensitivity(cases, windows=((1, 2), (1, 3), (2, 3)), stream=None, log=None, dump_dir=None):
    """Run each case of a sensitivity study (its own `steps`) and give C_Dave, C_Lrms and St over
    the statistics windows: (a, b) = from step a/b of the run to its end.  The first window is the
    study's main one.  With dump_dir, the per-step force series go to <dump_dir>/<name>.npz."""
    import os
    if dump_dir:
        os.makedirs(dump_dir, exist_ok=True)
    out = []
    for case in cases:
        r = run_series(case, case.steps, stream=stream, log=log)
        u, d = case.u_in[0], case.diameter
        ent = {"workload": case.name, "nx": case.nx, "ny": case.ny, "collision": case.collision,
               "storage": case.storage, "tau": case.tau, "eta": case.eta, "outlet": case.bc[1],
               "diameter": d, "cylinder_x": case.bodies[0]["cx"], "steps": case.steps,
               "status": int(r["status"]), "wall_s": round(r["wall_s"], 2),
               "mass_drift": float((r["mass"][-1] - r["mass"][0]) / r["mass"][0]), "windows": {}}
        for a, b in windows:
            first = case.steps * a // b
            ent["windows"][f"{first}-{case.steps}"] = A.wake_statistics(r["fx"], r["fy"], u, d, first=first)
        if dump_dir:
            np.savez_compressed(f"{dump_dir}/{case.name}.npz", mass=r["mass"], fx=r["fx"], fy=r["fy"])
        if log:
            w = ent["windows"][next(iter(ent["windows"]))]
            log(f"{case.name}: C_Dave {w['C_Dave']:.4f} C_Lrms {w['C_Lrms']:.4f} St {w['St']} "
                f"({r['wall_s']:.1f} s)")
        out.append(ent)
    return out


def body_force_regions(pop, mask, body_id, eta, usx=0.0, usy=0.0):
    """The penalization force the next step takes from the state `pop` ([9, ny, nx] FP64 f, as
    vplbm_get_populations gives it) on the nodes of body `body_id` at rest velocity (usx, usy),
    split into the surface layer (body nodes with a fluid node among their 8 neighbours) and the
    interior: f = -(j - rho u_s) / (eta + 1/2) after pull-streaming (Eqs. 8, 9, 17 with the
    well-conditioned form of the design notes), force on the body = -sum f.  Analysis only: the
    streaming here is plain periodic shifts, valid for bodies away from the lattice edges."""
    xi = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)])
    f = np.stack([np.roll(pop[a], (xi[a][1], xi[a][0]), axis=(0, 1)) for a in range(9)])
    rho = f.sum(axis=0)
    jx = np.tensordot(xi[:, 0], f, axes=1)
    jy = np.tensordot(xi[:, 1], f, axes=1)
    c = 1.0 / (eta + 0.5)
    fx = -(jx - rho * usx) * c
    fy = -(jy - rho * usy) * c
    solid = mask == body_id
    fluid = mask == 0
    near = np.zeros_like(fluid)
    for ex in (-1, 0, 1):
        for ey in (-1, 0, 1):
            near |= np.roll(fluid, (ey, ex), axis=(0, 1))
    surface = solid & near
    interior = solid & ~near
    # layers by distance to the fluid (1 = the surface layer, ..., 5 = five or more nodes in)
    layers = []
    reach = fluid.copy()
    left = solid.copy()
    for k in range(1, 6):
        grown = reach.copy()
        for ex in (-1, 0, 1):
            for ey in (-1, 0, 1):
                grown |= np.roll(reach, (ey, ex), axis=(0, 1))
        layer = left & grown if k < 5 else left
        layers.append((-float(fx[layer].sum()), -float(fy[layer].sum()), int(layer.sum())))
        left &= ~layer
        reach = grown
    return {"surface": (-float(fx[surface].sum()), -float(fy[surface].sum())),
            "interior": (-float(fx[interior].sum()), -float(fy[interior].sum())),
            "surface_nodes": int(surface.sum()), "interior_nodes": int(interior.sum()),
            "layers": layers}


def force_region_study(case, storages=("f64", "f32", "f16s", "f16sr"), steps=100_000,
                       first=50_000, every=500, stream=None, log=None):
    """Where the drag of reduced-precision storage differs from FP64: each storage runs `case`
    (a fixed body at rest), and from step `first` on, every `every` steps, the force the next
    step takes is split into the body's surface layer and interior (body_force_regions).  Returns
    per storage the time means of the drag (x) and lift (y) parts as force coefficients (Eq. 22),
    and the mean of the reduced per-step drag over the same steps."""
    u, d = case.u_in[0], case.diameter
    q = 0.5 * u * u * d
    out = {"workload": case.name, "steps": steps, "first": first, "every": every, "storages": {}}
    for st in storages:
        c = copy.copy(case)
        c.storage = st
        sim = B.Simulation(c, stream=stream, ring=every + 8)
        mask = None
        parts = {"surface": [], "interior": []}
        layers = []
        me_fx = []
        ring_fx = []
        sim.step(first)
        done = first
        nodes = None
        while done < steps:
            pop = sim.populations()
            if mask is None:
                mask = sim.mask()
            r = body_force_regions(pop, mask, 1, c.eta)
            nodes = (r["surface_nodes"], r["interior_nodes"])
            for k in parts:
                parts[k].append(r[k])
            layers.append([lx for lx, _, _ in r["layers"]])
            me_fx.append(sim.momentum_exchange()[0][0])
            sim.step(1)
            ring_fx.append(sim.force_series(done, 1)[0, 1])
            done += 1
            n = min(every - 1, steps - done)
            if n > 0:
                sim.step(n)
                done += n
        obs = sim.observables()
        sim.close()
        ent = {"status": int(obs["status"]), "samples": len(ring_fx),
               "surface_nodes": nodes[0], "interior_nodes": nodes[1],
               "C_D_reduced_at_samples": float(np.mean(ring_fx) / q)}
        for k, v in parts.items():
            a = np.array(v)
            ent[f"C_D_{k}"] = float(a[:, 0].mean() / q)
            ent[f"C_L_{k}_mean"] = float(a[:, 1].mean() / q)
        ent["C_D_split_total"] = ent["C_D_surface"] + ent["C_D_interior"]
        ent["C_D_by_layer"] = [float(v / q) for v in np.array(layers).mean(axis=0)]
        ent["C_D_momentum_exchange"] = float(np.mean(me_fx) / q)
        out["storages"][st] = ent
        if log:
            log(f"{case.name}/{st}: C_D surface {ent['C_D_surface']:.5f} interior "
                f"{ent['C_D_interior']:.6f} total {ent['C_D_split_total']:.5f} "
                f"(reduced {ent['C_D_reduced_at_samples']:.5f}, momentum exchange "
                f"{ent['C_D_momentum_exchange']:.5f}, {len(ring_fx)} samples); by layer "
                + " ".join(f"{v:.5f}" for v in ent["C_D_by_layer"]))
    return out
