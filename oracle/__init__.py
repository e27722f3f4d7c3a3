"""Python access to the FP64 CPU oracle of the VP-LBM step — TEST INFRASTRUCTURE ONLY.

The oracle (``vplbm_oracle.c``) is a plain FP64 implementation of Section 2 of arXiv:1812.05401
(Eqs. 2-18) with the boundary rules of Section 3.  Only ``tests/``, the smoke check and the
benchmark's CPU-baseline leg may import this module; the GPU library never does.

Array conventions: fields are ``[ny, nx]`` (x fastest); populations are ``[9, ny, nx]`` with the
direction numbering of Eq. 3.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

SRT, MRT = 0, 1
PERIODIC, VELOCITY, OUTFLOW, FREESLIP, CONVECTIVE = 0, 1, 2, 3, 4
DISK, RECT, DISK_OUTSIDE = 0, 1, 2
MAX_BODIES = 8


class Config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("collision", C.c_int32),
                ("tau", C.c_double), ("lambda_", C.c_double), ("eta", C.c_double),
                ("bc_xlo", C.c_int32), ("bc_xhi", C.c_int32), ("bc_ylo", C.c_int32),
                ("bc_yhi", C.c_int32), ("u_in_x", C.c_double), ("u_in_y", C.c_double),
                ("use_rates", C.c_int32), ("rates", C.c_double * 9)]


class Body(C.Structure):
    _fields_ = [("kind", C.c_int32), ("cx", C.c_double), ("cy", C.c_double), ("r", C.c_double),
                ("hx", C.c_double), ("hy", C.c_double), ("ux", C.c_double), ("uy", C.c_double),
                ("omega", C.c_double), ("ax", C.c_double), ("ay", C.c_double),
                ("freq", C.c_double)]


class Obs(C.Structure):
    _fields_ = [("step", C.c_int64), ("mass", C.c_double), ("fx", C.c_double * MAX_BODIES),
                ("fy", C.c_double * MAX_BODIES), ("fabs_sum", C.c_double * MAX_BODIES),
                ("nbodies", C.c_int32)]


_lib = None


def lib():
    """Load the oracle library, building it first if it is absent or older than its source."""
    global _lib
    if _lib is None:
        if (not os.path.exists(_build.LIB)
                or os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
            _build.build()
        L = C.CDLL(_build.LIB)
        dp = C.POINTER(C.c_double)
        L.orc_lattice.argtypes = [C.POINTER(C.c_int32), dp]
        L.orc_moment_matrix.argtypes = [dp]
        L.orc_feq.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        L.orc_forcing.argtypes = [C.c_double] * 4 + [dp]
        L.orc_meq.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        L.orc_mrt_rates.argtypes = [C.c_double, C.c_double, dp]
        L.orc_vp_macro.argtypes = [dp, C.c_int32, C.c_double, C.c_double, C.c_double, dp, dp, dp]
        L.orc_collide_srt.argtypes = [dp, C.c_double, dp, dp, C.c_double, dp]
        L.orc_collide_mrt.argtypes = [dp, C.c_double, dp, dp, dp, dp]
        L.orc_zou_he_inlet.argtypes = [dp, C.c_double, C.c_double]
        L.orc_body_state.argtypes = [C.POINTER(Body), C.c_double, dp, dp]
        L.orc_create.argtypes = [C.POINTER(Config)]
        L.orc_create.restype = C.c_void_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_bodies.argtypes = [C.c_void_p, C.POINTER(Body), C.c_int32, C.c_int32]
        L.orc_set_mask.argtypes = [C.c_void_p, C.POINTER(C.c_uint8)]
        L.orc_get_mask.argtypes = [C.c_void_p, C.POINTER(C.c_uint8)]
        L.orc_init_uniform.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double]
        L.orc_init_fields.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_set_populations.argtypes = [C.c_void_p, dp]
        L.orc_get_populations.argtypes = [C.c_void_p, dp]
        L.orc_pull_node.argtypes = [C.c_void_p, C.c_int32, C.c_int32, dp]
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_set_threads.argtypes = [C.c_void_p, C.c_int32]
        L.orc_set_threads.restype = C.c_int
        L.orc_get_threads.argtypes = [C.c_void_p]
        L.orc_get_threads.restype = C.c_int32
        L.orc_steps_done.argtypes = [C.c_void_p]
        L.orc_steps_done.restype = C.c_int64
        L.orc_get_obs.argtypes = [C.c_void_p, C.POINTER(Obs)]
        L.orc_get_fields.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_momentum_exchange.argtypes = [C.c_void_p, dp, dp]
        L.orc_residual.argtypes = [C.c_void_p, dp, dp]
        L.orc_residual.restype = C.c_double
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _vec(n):
    return np.zeros(n, dtype=np.float64)


# ---- constants and single-node operators --------------------------------------------------

def lattice():
    """(xi [9,2] int, w [9]) as the oracle uses them (Eqs. 3 and 5)."""
    xi = np.zeros(18, dtype=np.int32)
    w = _vec(9)
    lib().orc_lattice(xi.ctypes.data_as(C.POINTER(C.c_int32)), _dp(w))
    return xi.reshape(9, 2), w


def moment_matrix():
    m = _vec(81)
    lib().orc_moment_matrix(_dp(m))
    return m.reshape(9, 9)


def feq(rho, ux, uy):
    out = _vec(9)
    lib().orc_feq(rho, ux, uy, _dp(out))
    return out


def forcing(ux, uy, fx, fy):
    out = _vec(9)
    lib().orc_forcing(ux, uy, fx, fy, _dp(out))
    return out


def meq(rho, ux, uy):
    out = _vec(9)
    lib().orc_meq(rho, ux, uy, _dp(out))
    return out


def mrt_rates(tau, lam):
    out = _vec(9)
    lib().orc_mrt_rates(tau, lam, _dp(out))
    return out


def vp_macro(f, chi, us, eta):
    f = np.ascontiguousarray(f, dtype=np.float64)
    rho = C.c_double()
    u, fp = _vec(2), _vec(2)
    lib().orc_vp_macro(_dp(f), int(chi), us[0], us[1], eta, C.byref(rho), _dp(u), _dp(fp))
    return rho.value, u, fp


def collide_srt(f, rho, u, fpen, tau):
    f = np.ascontiguousarray(f, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    fpen = np.ascontiguousarray(fpen, dtype=np.float64)
    out = _vec(9)
    lib().orc_collide_srt(_dp(f), rho, _dp(u), _dp(fpen), tau, _dp(out))
    return out


def collide_mrt(f, rho, u, fpen, s):
    f = np.ascontiguousarray(f, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    fpen = np.ascontiguousarray(fpen, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    out = _vec(9)
    lib().orc_collide_mrt(_dp(f), rho, _dp(u), _dp(fpen), _dp(s), _dp(out))
    return out


def zou_he_inlet(f, ux, uy):
    f = np.array(f, dtype=np.float64)
    lib().orc_zou_he_inlet(_dp(f), ux, uy)
    return f


def make_body(kind=DISK, cx=0.0, cy=0.0, r=0.0, hx=0.0, hy=0.0, ux=0.0, uy=0.0, omega=0.0,
              ax=0.0, ay=0.0, freq=0.0):
    return Body(kind, cx, cy, r, hx, hy, ux, uy, omega, ax, ay, freq)


def body_state(body, t):
    c, v = _vec(2), _vec(2)
    lib().orc_body_state(C.byref(body), t, _dp(c), _dp(v))
    return c, v


# ---- whole-lattice simulation -------------------------------------------------------------

class OracleSim:
    """One lattice in the oracle.  Mirrors the GPU library's life cycle (create, mask, init,
    step, observe) so tests can drive both the same way."""

    def __init__(self, nx, ny, collision=SRT, tau=0.8, lam=3.0 / 16.0, eta=1e-7,
                 bc=(PERIODIC, PERIODIC, PERIODIC, PERIODIC), u_in=(0.0, 0.0), rates=None,
                 threads=1):
        cfg = Config()
        cfg.nx, cfg.ny, cfg.collision = nx, ny, collision
        cfg.tau, cfg.lambda_, cfg.eta = tau, lam, eta
        cfg.bc_xlo, cfg.bc_xhi, cfg.bc_ylo, cfg.bc_yhi = bc
        cfg.u_in_x, cfg.u_in_y = u_in
        if rates is not None:
            cfg.use_rates = 1
            for i in range(9):
                cfg.rates[i] = float(rates[i])
        h = lib().orc_create(C.byref(cfg))
        if not h:
            raise ValueError("oracle rejected the configuration")
        self.h = h
        self.nx, self.ny = nx, ny
        self.nbodies = 0
        self.set_threads(threads)

    def set_threads(self, n):
        """OpenMP threads for the node loops (0: every processor); the results are bitwise the
        same for every count.  Returns the count in use."""
        got = lib().orc_set_threads(self.h, int(n))
        if got < 0:
            raise ValueError("thread count must be >= 0")
        return got

    @property
    def threads(self):
        return lib().orc_get_threads(self.h)

    def close(self):
        if self.h:
            lib().orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_bodies(self, bodies, rasterize=True):
        arr = (Body * max(1, len(bodies)))(*bodies)
        if lib().orc_set_bodies(self.h, arr, len(bodies), 1 if rasterize else 0) != 0:
            raise ValueError("bad body table")
        self.nbodies = len(bodies)

    def set_mask(self, ids):
        ids = np.ascontiguousarray(ids, dtype=np.uint8)
        assert ids.shape == (self.ny, self.nx)
        if lib().orc_set_mask(self.h, ids.ctypes.data_as(C.POINTER(C.c_uint8))) != 0:
            raise ValueError("mask refers to a body that does not exist")

    def mask(self):
        ids = np.zeros((self.ny, self.nx), dtype=np.uint8)
        lib().orc_get_mask(self.h, ids.ctypes.data_as(C.POINTER(C.c_uint8)))
        return ids

    def init_uniform(self, rho0=1.0, ux0=0.0, uy0=0.0):
        lib().orc_init_uniform(self.h, rho0, ux0, uy0)

    def init_fields(self, rho, ux, uy):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        ux = np.ascontiguousarray(ux, dtype=np.float64)
        uy = np.ascontiguousarray(uy, dtype=np.float64)
        lib().orc_init_fields(self.h, _dp(rho), _dp(ux), _dp(uy))

    def set_populations(self, pop):
        pop = np.ascontiguousarray(pop, dtype=np.float64)
        assert pop.shape == (9, self.ny, self.nx)
        lib().orc_set_populations(self.h, _dp(pop))

    def populations(self):
        pop = np.zeros((9, self.ny, self.nx))
        lib().orc_get_populations(self.h, _dp(pop))
        return pop

    def pull_node(self, x, y):
        """Populations at node (x, y) after streaming and the edge rules, before collision."""
        f = _vec(9)
        lib().orc_pull_node(self.h, x, y, _dp(f))
        return f

    def step(self, n=1):
        lib().orc_step(self.h, int(n))

    @property
    def steps_done(self):
        return lib().orc_steps_done(self.h)

    def obs(self):
        o = Obs()
        lib().orc_get_obs(self.h, C.byref(o))
        nb = o.nbodies
        return {"step": o.step, "mass": o.mass, "fx": np.array(o.fx[:nb]),
                "fy": np.array(o.fy[:nb]), "fabs_sum": np.array(o.fabs_sum[:nb])}

    def momentum_exchange(self):
        """Per-body momentum-exchange force of the current state (fx, fy arrays)."""
        fx, fy = _vec(MAX_BODIES), _vec(MAX_BODIES)
        lib().orc_momentum_exchange(self.h, _dp(fx), _dp(fy))
        return fx[:self.nbodies], fy[:self.nbodies]

    def residual(self, ux_prev, uy_prev):
        """Relative L2 change of the fluid velocity against a previous field (Eq. 20 form)."""
        a = np.ascontiguousarray(ux_prev, dtype=np.float64)
        b = np.ascontiguousarray(uy_prev, dtype=np.float64)
        assert a.shape == b.shape == (self.ny, self.nx)
        return lib().orc_residual(self.h, _dp(a), _dp(b))

    def fields(self):
        rho = np.zeros((self.ny, self.nx))
        ux = np.zeros_like(rho)
        uy = np.zeros_like(rho)
        lib().orc_get_fields(self.h, _dp(rho), _dp(ux), _dp(uy))
        return rho, ux, uy
