"""Test helpers: build an oracle simulation from a seeded case description."""
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


def oracle_sim(case, rasterize=True, init=True):
    s = O.OracleSim(case.nx, case.ny, ORC_COLL[case.collision], tau=case.tau, lam=case.lam,
                    eta=case.eta, bc=tuple(ORC_BC[b] for b in case.bc), u_in=case.u_in)
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
