"""Seeded synthetic inputs for the VP-LBM workloads.

This module only draws and lays out inputs: grid sizes, relaxation parameters, obstacle tables,
initial density/velocity fields and request streams.  It holds none of the method's arithmetic
(no equilibria, no streaming, no collision, no penalization, no mask rasterization); the GPU
library and the test oracle each do that themselves from what is produced here.

Obstacles are plain dicts with the keys of the library's body record:
``kind`` ('disk', 'rect' or 'disk_outside'), ``cx, cy`` (centre at t = 0), ``r`` (radius),
``hx, hy`` (rectangle half-sides), ``ux, uy, omega`` (rigid velocity, u_s = U + omega e_z x (x - c)),
``ax, ay, freq`` (harmonic motion of the centre, c(t) = c0 + a sin(2 pi freq t)).
"""
from dataclasses import dataclass, field
import math
from typing import List, Optional, Tuple

import numpy as np

SRT, MRT = "srt", "mrt"
PERIODIC, VELOCITY, OUTFLOW, FREESLIP = "periodic", "velocity", "outflow", "freeslip"
CONVECTIVE = "convective"
CHANNEL = (VELOCITY, OUTFLOW, FREESLIP, FREESLIP)
CHANNEL_CONVECTIVE = (VELOCITY, CONVECTIVE, FREESLIP, FREESLIP)
ALL_PERIODIC = (PERIODIC, PERIODIC, PERIODIC, PERIODIC)
GINZBURG_LAMBDA = 3.0 / 16.0   # Section 2.1.2: the value used with s_n = 1/tau


def body(kind="disk", cx=0.0, cy=0.0, r=0.0, hx=0.0, hy=0.0, ux=0.0, uy=0.0, omega=0.0,
         ax=0.0, ay=0.0, freq=0.0) -> dict:
    return dict(kind=kind, cx=float(cx), cy=float(cy), r=float(r), hx=float(hx), hy=float(hy),
                ux=float(ux), uy=float(uy), omega=float(omega), ax=float(ax), ay=float(ay),
                freq=float(freq))


def tau_from_reynolds(u: float, length: float, re: float) -> float:
    """Relaxation time for a target Reynolds number: nu = U L / Re and tau = 3 nu + 1/2 (Eq. 6)."""
    return 0.5 + 3.0 * u * length / re


@dataclass
class Case:
    """One simulation: what the user of the library supplies."""
    name: str
    nx: int
    ny: int
    collision: str = MRT
    storage: str = "f32"
    tau: float = 0.8
    lam: float = GINZBURG_LAMBDA
    eta: float = 1e-7
    bc: Tuple[str, str, str, str] = ALL_PERIODIC
    u_in: Tuple[float, float] = (0.0, 0.0)
    bodies: List[dict] = field(default_factory=list)
    rho0: float = 1.0
    u0: Tuple[float, float] = (0.0, 0.0)
    steps: int = 1000
    diameter: Optional[float] = None   # reference length for force coefficients

    @property
    def nodes(self) -> int:
        return self.nx * self.ny


# ---- the five workloads -------------------------------------------------------------------

def taylor_couette_128() -> Case:
    """Rotating inner disk r = 20 (tangential speed 0.05) inside a fixed annulus r >= 50, centred
    on a 128 x 128 periodic lattice, SRT tau = 0.8, 1/eta = 1, FP64, 5000 steps."""
    c = 63.5
    return Case("taylor_couette_128", 128, 128, collision=SRT, storage="f64", tau=0.8, eta=1.0,
                bc=ALL_PERIODIC,
                bodies=[body("disk", c, c, r=20.0, omega=0.05 / 20.0),
                        body("disk_outside", c, c, r=50.0)],
                steps=5000)


def cylinder_wake(nx=2048, ny=512, d=64.0, x0=512.0, re=200.0, u=0.05, storage="f32",
                  steps=100_000) -> Case:
    """Fixed disk of diameter d in a channel: Zou-He inlet u, zero-gradient outflow, free-slip
    walls, VP-MRT with Lambda = 3/16.  The disk centre sits at y = ny/2, half a node off the
    channel's mid-plane, which breaks the symmetry deterministically and starts shedding."""
    return Case(f"cylinder_wake_{nx}x{ny}", nx, ny, collision=MRT, storage=storage,
                tau=tau_from_reynolds(u, d, re), bc=CHANNEL, u_in=(u, 0.0),
                bodies=[body("disk", x0, ny / 2.0, r=d / 2.0)], u0=(u, 0.0), steps=steps,
                diameter=d)


def cylinder_wake_2048x512() -> Case:
    return cylinder_wake()


def cylinder_wake_8192x2048(storage="f16s") -> Case:
    """The 2048 x 512 case's parameters in a 8192 x 2048 channel (disk D = 64 at x = 512)."""
    return cylinder_wake(8192, 2048, storage=storage)


def oscillating_cylinder_8192x2048(steps=200_000) -> Case:
    """Disk D = 96 oscillating across the flow, amplitude 0.2 D, frequency 0.2 u/D, Re = 300."""
    u, d = 0.05, 96.0
    c = cylinder_wake(8192, 2048, d=d, x0=1024.0, re=300.0, u=u, steps=steps)
    c.name = "oscillating_cylinder_8192x2048"
    c.bodies = [body("disk", 1024.0, 1024.0, r=d / 2.0, ay=0.2 * d, freq=0.2 * u / d)]
    return c


def paper_cylinder_re500(storage="f32", steps=500_000) -> Case:
    """The paper's bluff-body case (Section 3.3): a 30 D x 10 D channel resolved by 6048 x 2016
    nodes, D = 201 nodes, the cylinder 25 D from the outlet, inlet speed 0.05, SRT tau = 0.56
    (Re = 0.05 * 201 / ((0.56 - 1/2)/3) = 502.5), symmetry (free-slip) planes above and below,
    convective outlet, eta = 1e-7.  The centre sits at y = ny/2, half a node off the mid-plane."""
    nx, ny, d = 6048, 2016, 201.0
    return Case("paper_cylinder_re500", nx, ny, collision=SRT, storage=storage, tau=0.56, eta=1e-7,
                bc=CHANNEL_CONVECTIVE, u_in=(0.05, 0.0), u0=(0.05, 0.0),
                bodies=[body("disk", nx - 25 * d, ny / 2.0, r=d / 2.0)], steps=steps, diameter=d)


def paper_cylinder_variant(label, storage="f32", upstream=5.0, downstream=25.0, height=10.0,
                           scale=1.0, collision=SRT, eta=1e-7, outlet=CONVECTIVE) -> Case:
    """The paper's Re = 500 cylinder (paper_cylinder_re500) with one setting changed, for a
    sensitivity study: the inlet `upstream` diameters before the cylinder centre (5 in the paper;
    the paper's lattice puts it 1023 nodes = 5.09 D from the inlet, kept for every variant), the
    outlet `downstream` diameters after it (25), the channel `height` in diameters (10), the
    resolution (`scale` times 201 nodes per diameter, Re and U kept, so tau follows Eq. 6), the
    collision (SRT in the paper; MRT with Lambda = 3/16), eta, and the outlet rule (convective,
    R13, or zero-gradient).  Steps and the statistics window scale with D / U."""
    d = 201.0 * scale
    re = 0.05 * 201.0 / ((0.56 - 0.5) / 3.0)          # 502.5, the paper's case
    up = int(round(1023 * scale + (upstream - 5.0) * d))
    nx = up + int(round(downstream * d))
    ny = int(round(2016 * scale * height / 10.0))
    bc = (VELOCITY, CONVECTIVE if outlet == CONVECTIVE else OUTFLOW, FREESLIP, FREESLIP)
    return Case(f"paper_cylinder_re500_{label}", nx, ny, collision=collision, storage=storage,
                tau=tau_from_reynolds(0.05, d, re), eta=eta, bc=bc, u_in=(0.05, 0.0),
                u0=(0.05, 0.0), bodies=[body("disk", up, ny / 2.0, r=d / 2.0)],
                steps=int(round(600_000 * scale)), diameter=d)


def paper_cylinder_sensitivity(storage="f32") -> List[Case]:
    """The variants of the Re = 500 study, the paper's own setup first."""
    return [paper_cylinder_variant("base", storage),
            paper_cylinder_variant("zero_gradient_outlet", storage, outlet=OUTFLOW),
            paper_cylinder_variant("eta_1e-5", storage, eta=1e-5),
            paper_cylinder_variant("eta_1e-3", storage, eta=1e-3),
            paper_cylinder_variant("inlet_10d", storage, upstream=10.0),
            paper_cylinder_variant("outlet_40d", storage, downstream=40.0),
            paper_cylinder_variant("mrt", storage, collision=MRT),
            paper_cylinder_variant("half_resolution", storage, scale=0.5),
            paper_cylinder_variant("height_20d", storage, height=20.0),
            paper_cylinder_variant("inlet_20d", storage, upstream=20.0),
            paper_cylinder_variant("inlet_10d_height_20d", storage, upstream=10.0, height=20.0),
            paper_cylinder_variant("half_resolution_mrt", storage, scale=0.5, collision=MRT),
            paper_cylinder_variant("inlet_20d_height_40d", storage, upstream=20.0, height=40.0)]


# ---- random inputs for parity tests ---------------------------------------------------------

def random_fields(nx: int, ny: int, seed: int, rho_amp=0.02, u_amp=0.03, u_mean=(0.0, 0.0)):
    """Density ~ 1 + U(-rho_amp, rho_amp) and velocity ~ u_mean + U(-u_amp, u_amp) per node."""
    r = np.random.default_rng(seed)
    rho = 1.0 + r.uniform(-rho_amp, rho_amp, (ny, nx))
    ux = u_mean[0] + r.uniform(-u_amp, u_amp, (ny, nx))
    uy = u_mean[1] + r.uniform(-u_amp, u_amp, (ny, nx))
    return rho, ux, uy


def random_bodies(nx: int, ny: int, seed: int, n: int, moving=False, rmin=2.0, rmax=None):
    """Up to n disks/rectangles with random centres and sizes inside the lattice, their boxes
    (swept boxes when moving) at least two nodes apart.  The solid velocity is always consistent
    with the body's own motion, so no mask forces flow through a fixed region or into another
    body: disks spin about their centre (|omega r| <= 0.02), rectangles are at rest, and with
    ``moving`` every body also oscillates (velocity amplitude <= 0.025)."""
    r = np.random.default_rng(seed)
    rmax = rmax if rmax is not None else max(rmin + 1.0, min(nx, ny) / 6.0)
    out, boxes = [], []
    for k in range(n):
        for _attempt in range(200):
            kind = "disk" if r.random() < 0.5 else "rect"
            rad = min(r.uniform(rmin, rmax), min(nx, ny) / 2.0 - 2.0)
            cx = r.uniform(rad + 1, nx - rad - 2)
            cy = r.uniform(rad + 1, ny - rad - 2)
            omega = r.uniform(-0.02, 0.02) / max(rad, 1.0) if kind == "disk" else 0.0
            b = body(kind, cx, cy, r=rad, hx=rad * r.uniform(0.5, 1.0), hy=rad * r.uniform(0.5, 1.0),
                     omega=omega)
            if moving:
                b.update(ax=r.uniform(-2, 2), ay=r.uniform(-2, 2), freq=r.uniform(0.0005, 0.002))
            ex = (rad if kind == "disk" else b["hx"]) + abs(b["ax"]) + 1.0
            ey = (rad if kind == "disk" else b["hy"]) + abs(b["ay"]) + 1.0
            box = (cx - ex, cx + ex, cy - ey, cy + ey)
            if all(box[1] < o[0] or o[1] < box[0] or box[3] < o[2] or o[3] < box[2] for o in boxes):
                out.append(b)
                boxes.append(box)
                break
    return out


# ---- the serving workload ---------------------------------------------------------------------

@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the stream
    case: Case


def column_blockage(bodies, n) -> float:
    """Largest fraction of a lattice column (x = const) that the bodies' chords cover, overlaps
    counted twice (an upper bound)."""
    x = np.arange(n, dtype=np.float64)
    cover = np.zeros(n)
    for b in bodies:
        if b["kind"] == "disk":
            cover += 2.0 * np.sqrt(np.maximum(b["r"] ** 2 - (x - b["cx"]) ** 2, 0.0))
        else:
            cover += np.where(np.abs(x - b["cx"]) <= b["hx"], 2.0 * b["hy"], 0.0)
    return float(cover.max() / n)


def serving_requests(n=256, seed_arrivals=1812, seed_geometry=5401, rate_per_s=1.0,
                     nmin=128, nmax=1024, nstep=32, steps_range=(1000, 20000),
                     re_range=(50.0, 500.0), u=0.05) -> List[Request]:
    """Poisson arrivals of square VP-MRT channel simulations, FP32, 1-8 random disks and
    rectangles (radius or half-side 8 to min(64, N/8)), Re 50-500, 1k-20k steps.  Each obstacle
    lies in x in [max(N/8, r+4), 5N/8], y in [r+6, N-r-7]; draws with more than 20% solid area,
    a column more than 40% blocked (column_blockage) or tau < 0.56 are redrawn.  (With radii up
    to N/2, obstacles reaching the inlet or two nodes from a wall, crowded columns and tau down
    to 0.51, 30 of the 256 default requests went unstable.)"""
    ra = np.random.default_rng(seed_arrivals)
    rg = np.random.default_rng(seed_geometry)
    gaps = ra.exponential(1.0 / rate_per_s, n)
    arrivals = np.cumsum(gaps) - gaps[0]
    sizes = np.arange(nmin, nmax + 1, nstep)
    out = []
    for i in range(n):
        while True:
            N = int(rg.choice(sizes))
            k = int(rg.integers(1, 9))
            bodies, area, rmax = [], 0.0, 0.0
            for _ in range(k):
                rad = float(rg.uniform(8, min(64.0, N / 8.0)))
                kind = "disk" if rg.random() < 0.5 else "rect"
                cx = float(rg.uniform(max(N / 8, rad + 4), 5 * N / 8))
                cy = float(rg.uniform(rad + 6, N - rad - 7))
                bodies.append(body(kind, cx, cy, r=rad, hx=rad, hy=rad))
                area += math.pi * rad * rad if kind == "disk" else 4 * rad * rad
                rmax = max(rmax, rad)
            re = float(rg.uniform(*re_range))
            tau = tau_from_reynolds(u, 2 * rmax, re)
            steps = int(rg.integers(steps_range[0], steps_range[1] + 1))
            if area <= 0.2 * N * N and tau >= 0.56 and column_blockage(bodies, N) <= 0.4:
                break
        c = Case(f"req{i}", N, N, collision=MRT, storage="f32", tau=tau, bc=CHANNEL,
                 u_in=(u, 0.0), bodies=bodies, u0=(u, 0.0), steps=steps, diameter=2 * rmax)
        out.append(Request(i, float(arrivals[i]), c))
    return out
