"""Test helpers: build an oracle simulation from a seeded case description."""
import math
import os

import numpy as np

import oracle as O
from paper_1812_05401_amd import inputs as I

ORC_COLL = {I.SRT: O.SRT, I.MRT: O.MRT}
ORC_BC = {I.PERIODIC: O.PERIODIC, I.VELOCITY: O.VELOCITY, I.OUTFLOW: O.OUTFLOW,
          I.FREESLIP: O.FREESLIP, I.CONVECTIVE: O.CONVECTIVE}
ORC_KIND = {"disk": O.DISK, "rect": O.RECT, "disk_outside": O.DISK_OUTSIDE}


def orc_body(b):
    return O.make_body(ORC_KIND[b["kind"]], b["cx"], b["cy"], b["r"], b["hx"], b["hy"], b["ux"],
                       b["uy"], b["omega"], b["ax"], b["ay"], b["freq"])


def host_threads():
    """Threads the oracle may use here: the processors this process may run on, at most the
    OMP_NUM_THREADS the environment sets (the share of the host's CPUs a job is given)."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(n, 1)


def oracle_sim(case, rasterize=True, init=True, threads=1):
    s = O.OracleSim(case.nx, case.ny, ORC_COLL[case.collision], tau=case.tau, lam=case.lam,
                    eta=case.eta, bc=tuple(ORC_BC[b] for b in case.bc), u_in=case.u_in,
                    threads=threads)
    if case.bodies:
        s.set_bodies([orc_body(b) for b in case.bodies], rasterize=rasterize)
    if init:
        s.init_uniform(case.rho0, *case.u0)
    return s


def rel_err(a, b):
    """max |a - b| / max |b| over all entries."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def gpu_sim(case, storage=None, device_mask=True, init=True, reduce=True, ring=0):
    """A GPU simulation through the C ABI for a case (torch supplies the stream)."""
    from paper_1812_05401_amd import binding as B
    kw = {}
    if storage is not None:
        kw["storage"] = storage
    import copy
    c = copy.copy(case)
    if storage is not None:
        c.storage = storage
    s = B.Simulation(c, stream="torch", reduce=reduce, ring=ring, device_mask=device_mask)
    return s


def force_scale(orc_obs):
    """Scale for comparing body forces: the summed magnitude of the penalization force."""
    return max(float(np.sum(orc_obs["fabs_sum"])), 1e-300)


def couette_l2(ux, uy, ids, L, R1, R2, ud):
    """Relative L2 error (Eq. 20) of a velocity field against Taylor-Couette flow (Eq. 21) between
    a disk of radius R1 turning at surface speed ud and a fixed ring of radius R2, both centred on
    the L x L lattice, over the fluid nodes: (vector error, error of the y component)."""
    c = (L - 1) / 2
    y, x = np.mgrid[0:L, 0:L]
    dx, dy = x - c, y - c
    r = np.hypot(dx, dy)
    ut = -ud * R1 * r / (R2 ** 2 - R1 ** 2) + ud * R1 * R2 ** 2 / ((R2 ** 2 - R1 ** 2) * r)
    ax, ay = -ut * dy / r, ut * dx / r
    fluid = ids == 0
    err_vec = math.sqrt(np.sum(((ux - ax) ** 2 + (uy - ay) ** 2)[fluid])
                        / np.sum((ax ** 2 + ay ** 2)[fluid]))
    err_v = math.sqrt(np.sum(((uy - ay) ** 2)[fluid]) / np.sum((ay ** 2)[fluid]))
    return err_vec, err_v
