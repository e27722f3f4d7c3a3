"""Parameter sweeps of Section 3 as a batched workload: many small simulations run together in
the serving pool, each reduced to the relative L2 error of Eq. 20 against its analytic profile.

* plane shear between penalized plates (Eq. 19): error against tau for SRT and against Lambda for
  MRT (Fig. 3); the paper reports it practically vanishes at tau = 1/2 + sqrt(6)/4 (SRT) and at
  Lambda = 3/8 (MRT, any tau);
* Taylor-Couette flow between a rotating inner and a fixed outer cylinder (Eq. 21): error of the
  vertical velocity against Lambda at tau = 0.7 and tau = 10 (Fig. 12; the paper runs tau = 10 at
  Lambda = 0.0016), and against the grid resolution of Table 1 (Fig. 17).

Readings: the shear flow is x-invariant, so the 200-node-long domain of the paper is run 64 nodes
long (periodic); the plates are the rows y <= e and y >= e + H (reading R11 of the design notes).
For Table 1 the radii scale with the box (R2 = 0.35 L, R1 = R2 - Ngrid), which reproduces the
paper's R1 = 45, R2 = 70 at L = 200.
"""
import math
from dataclasses import dataclass
from typing import List

import numpy as np

from . import analysis as A
from . import inputs as I

SHEAR_UD, SHEAR_E, SHEAR_H, SHEAR_NY = 0.01, 50.0, 100.0, 200


def relax_steps(gap, tau, efolds=16.0, minimum=2000, maximum=600_000):
    """Steps for the slowest viscous mode across a gap to decay by e^efolds: the diffusion time
    gap^2 / (pi^2 nu) per e-fold with nu = (tau - 1/2)/3 (Eq. 6)."""
    nu = (tau - 0.5) / 3.0
    return int(min(maximum, max(minimum, efolds * gap * gap / (math.pi ** 2 * nu))))


@dataclass
class SweepPoint:
    label: str
    params: dict
    case: I.Case
    error_of: object      # callable(rho, ux, uy) -> float
    other_errors: object = None   # callable(rho, ux, uy) -> dict of other error measures


def shear_case(collision, tau, lam=0.375, steps=None, nx=64, storage="f64"):
    ud, e, H, ny = SHEAR_UD, SHEAR_E, SHEAR_H, SHEAR_NY
    steps = steps or relax_steps(H, tau)
    bodies = [I.body("rect", (nx - 1) / 2, e / 2, hx=nx, hy=e / 2, ux=-ud),
              I.body("rect", (nx - 1) / 2, (e + H + ny - 1) / 2, hx=nx, hy=(ny - 1 - e - H) / 2, ux=ud)]
    case = I.Case(f"shear_{collision}_tau{tau:g}_lam{lam:g}", nx, ny, collision=collision,
                  storage=storage, tau=tau, lam=lam, eta=1e-7, bc=I.ALL_PERIODIC, bodies=bodies,
                  steps=steps)
    y = np.arange(ny)
    ua = (2 * ud / H) * (y - e) - ud                        # Eq. 19
    fluid_rows = (y > e) & (y < e + H)

    def err(rho, ux, uy):
        fluid = np.broadcast_to(fluid_rows[:, None], ux.shape)
        return A.l2_error(ux, np.broadcast_to(ua[:, None], ux.shape), fluid)
    return SweepPoint(case.name, {"collision": collision, "tau": tau, "lambda": lam}, case, err)


def couette_case(collision, tau, lam, L=200, ngrid=25, ud=0.01, steps=None, storage="f64",
                 centre=None):
    """Taylor-Couette flow (Eq. 21) between a disk turning at surface speed ud and a fixed ring,
    centred at (centre, centre): (L - 1)/2 by default (reading R5 of the design notes), L/2 as an
    alternative staircase.  Besides the L2 error of v over the fluid annulus (the measure of
    Figs 11, 12 and 17), the point reports the same without the staircase layer (fluid nodes with
    a solid neighbour), along the line y = L/2 of Fig. 13, and of the velocity vector."""
    steps = steps or relax_steps(ngrid, tau)
    R2 = 0.35 * L
    R1 = R2 - ngrid
    c = (L - 1) / 2 if centre is None else centre
    bodies = [I.body("disk", c, c, r=R1, omega=ud / R1), I.body("disk_outside", c, c, r=R2)]
    tag = "" if centre is None else f"_c{c:g}"
    case = I.Case(f"couette_{collision}_L{L}_tau{tau:g}_lam{lam:g}{tag}", L, L, collision=collision,
                  storage=storage, tau=tau, lam=lam, eta=1e-7, bc=I.ALL_PERIODIC, bodies=bodies,
                  steps=steps)
    yy, xx = np.mgrid[0:L, 0:L]
    dx, dy = xx - c, yy - c
    r = np.hypot(dx, dy)
    with np.errstate(divide="ignore", invalid="ignore"):
        ut = -ud * R1 * r / (R2 ** 2 - R1 ** 2) + ud * R1 * R2 ** 2 / ((R2 ** 2 - R1 ** 2) * r)  # Eq. 21
        vy = ut * dx / r
        vx = -ut * dy / r
    fluid = (r > R1) & (r < R2)
    near = np.zeros_like(fluid)
    for ex in (-1, 0, 1):
        for ey in (-1, 0, 1):
            near |= np.roll(~fluid, (ey, ex), axis=(0, 1))
    inner = fluid & ~near
    line = np.zeros_like(fluid)
    line[int(round(L / 2)), :] = True
    line &= fluid

    def err(rho, ux, uy):
        return A.l2_error(uy, vy, fluid)

    def others(rho, ux, uy):
        return {"l2_v_without_staircase_layer": float(A.l2_error(uy, vy, inner)),
                "l2_v_line_y_half": float(A.l2_error(uy, vy, line)),
                "l2_vector": float(A.l2_error(np.stack([ux, uy]), np.stack([vx, vy]),
                                              np.stack([fluid, fluid])))}
    return SweepPoint(case.name, {"collision": collision, "tau": tau, "lambda": lam, "L": L,
                                  "Ngrid": ngrid, "centre": c}, case, err, others)


def fig3_shear():
    pts = [shear_case("srt", t) for t in (0.6, 0.8, 1.0, 0.5 + math.sqrt(6) / 4, 1.3, 1.6, 2.0)]
    for tau in (0.7, 1.5, 10.0):
        pts += [shear_case("mrt", tau, lam) for lam in (0.1, 3 / 16, 0.3, 0.375, 0.5, 1.0)]
    return pts


def fig12_couette():
    pts = [couette_case("mrt", 0.7, lam) for lam in (0.01, 0.05, 0.1, 3 / 16, 0.375, 0.75)]
    pts += [couette_case("mrt", 10.0, lam) for lam in (0.0005, 0.0016, 0.005, 0.02, 0.06, 0.1, 0.2,
                                                       0.375)]
    pts += [couette_case("srt", t, 0.0) for t in (0.7, 1.0, 10.0)]
    return pts


def fig12_readings(steps_scale=1):
    """Readings of Fig. 12 at tau = 10 and 0.7: a dense Lambda sweep near zero, the disk centred
    at (L - 1)/2 and at L/2, each point reporting every error measure of couette_case; with
    steps_scale the runs go steps_scale times longer than the viscous relaxation estimate (at
    tau = 10 and Lambda = 0.0016 the odd rate is 1.9993, whose non-hydrodynamic modes decay by
    only 0.07% per step)."""
    lams = (0.0005, 0.0016, 0.005, 0.01, 0.02, 0.04, 0.06, 0.08, 0.1, 0.14, 3 / 16, 0.375)
    pts = []
    for tau in (10.0, 0.7):
        steps = relax_steps(25, tau) * steps_scale
        for c in (None, 100.0):
            pts += [couette_case("mrt", tau, lam, steps=steps, centre=c) for lam in lams]
    return pts


def table1_grids():
    """Couette at the resolutions of Table 1, MRT tau = 0.7, Lambda = 3/16 and 3/8."""
    pts = []
    for L, ng in ((200, 25), (400, 50), (600, 75), (800, 100), (800, 125)):
        for lam in (3 / 16, 0.375):
            pts.append(couette_case("mrt", 0.7, lam, L=L, ngrid=ng))
    return pts


def fig5_convergence(max_steps=600_000):
    """Iterations to convergence of the plane shear (Figs 5-7): each point runs until its
    residual over 1000 steps is below 1e-12 (the pool's early stop) or max_steps.  The paper finds
    SRT tau = 1/2 + sqrt(6)/4 and MRT Lambda = 3/8 at that tau the fastest to an error near zero."""
    opt = 0.5 + math.sqrt(6) / 4
    pts = [shear_case("srt", t, steps=max_steps) for t in (0.6, 0.8, 1.0, opt, 1.3, 1.6, 2.0)]
    pts += [shear_case("mrt", t, 0.375, steps=max_steps) for t in (0.7, opt, 1.5, 10.0)]
    return pts


def fig14_convergence(max_steps=200_000):
    """Iterations to convergence of the Taylor-Couette flow (Figs 14-15), residual over 1000
    steps below 1e-5: MRT at tau = 0.7 (Lambda = 0.1, 3/16) and tau = 10 (Lambda = 0.0016, the
    paper's choice, and 0.06), SRT at tau = 0.7, 1 and 10."""
    pts = [couette_case("mrt", 0.7, lam, steps=max_steps) for lam in (0.1, 3 / 16)]
    pts += [couette_case("mrt", 10.0, lam, steps=max_steps) for lam in (0.0016, 0.06)]
    pts += [couette_case("srt", t, 0.0, steps=max_steps) for t in (0.7, 1.0, 10.0)]
    return pts


CONVERGENCE_STOP = {"fig5": (1e-12, 1000), "fig14": (1e-5, 1000)}


def run(points: List[SweepPoint], budget_bytes=8 << 30, max_slots=256, steps_per_launch=256,
        stop=None):
    """Run every point through the pool at once, for its step count or, with stop = (tol,
    every), until its convergence residual over `every` steps falls below tol.  Returns one
    record per point: label, parameters, L2 error, status, steps run and last residual."""
    from . import binding as B
    pool = B.Pool(budget_bytes, max_slots=max_slots, steps_per_launch=steps_per_launch)
    ids = {pool.submit(p.case, p.case.steps, keep_fields=True, stop=stop): p for p in points}
    out = {}
    while len(out) < len(ids):
        pool.advance()
        for rid, p in ids.items():
            if rid in out:
                continue
            st, done = pool.status(rid)
            if st in (B.DONE, B.FAILED):
                res = pool.residual(rid)
                obs, (rho, ux, uy) = pool.result(rid, fields=True)
                out[rid] = {"label": p.label, **p.params, "l2_error": float(p.error_of(rho, ux, uy)),
                            "status": int(obs["status"]), "steps": int(done),
                            "residual": None if math.isinf(res) else float(res)}
                if p.other_errors:
                    out[rid].update(p.other_errors(rho, ux, uy))
    pool.close()
    return [out[r] for r in ids]
