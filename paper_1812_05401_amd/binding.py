"""ctypes binding of the C ABI in include/vplbm.h (argument marshalling only).

Every function here calls the HIP library ``libvplbm.so``; there is no other compute path.  If
the library is missing, every call raises.  Function names follow the C entry points; the
``Simulation`` class wraps one handle.

Array conventions: fields are numpy ``[ny, nx]`` FP64 (x fastest); populations ``[9, ny, nx]``.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

ABI_VERSION = 1
MAX_BODIES = 8
RING_WIDTH = 1 + 2 * MAX_BODIES

OK, EINVAL, ENOMEM, EHIP, EUNSTABLE, EBUDGET, ESTATE = 0, -1, -2, -3, -4, -5, -6
SRT, MRT = 0, 1
F64, F32, F16S, BF16S, F32D, F16SR, BF16SR = 0, 1, 2, 3, 4, 5, 6
PERIODIC, VELOCITY, OUTFLOW, FREESLIP, CONVECTIVE = 0, 1, 2, 3, 4
DISK, RECT, DISK_OUTSIDE = 0, 1, 2

STORAGE = {"f64": F64, "f32": F32, "f16s": F16S, "bf16s": BF16S, "f32d": F32D, "f16sr": F16SR,
           "bf16sr": BF16SR,
           # the 16-bit formats by their plain names are the stochastically rounded ones: they keep
           # the mass of long runs, and drag and St within 1% of FP64 on large lattices (bfloat16
           # rounded to nearest is not usable for force statistics)
           "f16": F16SR, "bf16": BF16SR}
COLLISION = {"srt": SRT, "mrt": MRT}
BC = {"periodic": PERIODIC, "velocity": VELOCITY, "outflow": OUTFLOW, "freeslip": FREESLIP,
      "convective": CONVECTIVE}
SHAPE = {"disk": DISK, "rect": RECT, "disk_outside": DISK_OUTSIDE}


class VplbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"vplbm error {code}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("collision", C.c_int32), ("storage", C.c_int32), ("tau", C.c_double),
                ("lambda_", C.c_double), ("eta", C.c_double), ("rho0", C.c_double),
                ("ux0", C.c_double), ("uy0", C.c_double), ("bc_xlo", C.c_int32),
                ("bc_xhi", C.c_int32), ("bc_ylo", C.c_int32), ("bc_yhi", C.c_int32),
                ("u_in_x", C.c_double), ("u_in_y", C.c_double), ("reduce", C.c_int32),
                ("ring", C.c_int32), ("stream", C.c_void_p)]


class Body(C.Structure):
    _fields_ = [("kind", C.c_int32), ("cx", C.c_double), ("cy", C.c_double), ("r", C.c_double),
                ("hx", C.c_double), ("hy", C.c_double), ("ux", C.c_double), ("uy", C.c_double),
                ("omega", C.c_double), ("ax", C.c_double), ("ay", C.c_double),
                ("freq", C.c_double)]


class PoolConfig(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("budget_bytes", C.c_uint64), ("max_slots", C.c_int32),
                ("steps_per_launch", C.c_int32), ("stream", C.c_void_p)]


class Obs(C.Structure):
    _fields_ = [("step", C.c_int64), ("mass", C.c_double), ("fx", C.c_double * MAX_BODIES),
                ("fy", C.c_double * MAX_BODIES), ("nbodies", C.c_int32), ("status", C.c_int32)]


# (name, restype, argtypes) of every entry point declared in include/vplbm.h
_dp = C.POINTER(C.c_double)
SIGNATURES = [
    ("vplbm_create", C.c_int, [C.POINTER(Config), C.POINTER(C.c_void_p)]),
    ("vplbm_set_mask", C.c_int, [C.c_void_p, C.POINTER(C.c_uint8), C.POINTER(Body), C.c_int32]),
    ("vplbm_step", C.c_int, [C.c_void_p, C.c_int64]),
    ("vplbm_observables", C.c_int, [C.c_void_p, C.POINTER(Obs), _dp, _dp, _dp]),
    ("vplbm_destroy", C.c_int, [C.c_void_p]),
    ("vplbm_last_error", C.c_char_p, []),
    ("vplbm_init_fields", C.c_int, [C.c_void_p, _dp, _dp, _dp]),
    ("vplbm_get_populations", C.c_int, [C.c_void_p, _dp]),
    ("vplbm_set_populations", C.c_int, [C.c_void_p, _dp, C.c_int64]),
    ("vplbm_get_mask", C.c_int, [C.c_void_p, C.POINTER(C.c_uint8)]),
    ("vplbm_force_series", C.c_int, [C.c_void_p, C.c_int64, C.c_int64, _dp]),
    ("vplbm_momentum_exchange", C.c_int, [C.c_void_p, _dp, _dp]),
    ("vplbm_momentum_exchange_noalloc", C.c_int, [C.c_void_p, C.c_void_p]),
    ("vplbm_residual", C.c_int, [C.c_void_p, _dp]),
    ("vplbm_steps_done", C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("vplbm_steps_per_launch", C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    ("vplbm_stream", C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
    ("vplbm_bytes_per_update", C.c_int, [C.c_int32, C.POINTER(C.c_int64)]),
    ("vplbm_pool_create", C.c_int, [C.POINTER(PoolConfig), C.POINTER(C.c_void_p)]),
    ("vplbm_pool_submit", C.c_int, [C.c_void_p, C.POINTER(Config), C.POINTER(Body), C.c_int32,
                                     C.c_int64, C.c_int32, C.POINTER(C.c_int64)]),
    ("vplbm_pool_set_stop", C.c_int, [C.c_void_p, C.c_int64, C.c_double, C.c_int64]),
    ("vplbm_pool_set_admission", C.c_int, [C.c_void_p, C.c_uint64]),
    ("vplbm_pool_cancel", C.c_int, [C.c_void_p, C.c_int64]),
    ("vplbm_pool_residual", C.c_int, [C.c_void_p, C.c_int64, _dp]),
    ("vplbm_pool_advance", C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32)]),
    ("vplbm_pool_status", C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    ("vplbm_pool_result", C.c_int, [C.c_void_p, C.c_int64, C.POINTER(Obs), _dp, _dp, _dp]),
    ("vplbm_pool_bytes_needed", C.c_int, [C.POINTER(Config), C.POINTER(C.c_uint64)]),
    ("vplbm_pool_destroy", C.c_int, [C.c_void_p]),
]
QUEUED, RUNNING, DONE, FAILED, CANCELLED = 0, 1, 2, 3, 4

_lib = None


def library_path():
    """The in-tree build, or the build named by VPLBM_LIB (another build of the same sources,
    e.g. for A/B timing of kernel variants)."""
    return os.environ.get("VPLBM_LIB") or _build.LIB


def load():
    """Load libvplbm.so (built in-tree by ``python -m paper_1812_05401_amd.build``)."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built: run python -m paper_1812_05401_amd.build")
        L = C.CDLL(path)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error():
    return load().vplbm_last_error().decode()


def check(rc):
    if rc != OK:
        raise VplbmError(rc, last_error())
    return rc


def _ptr(a, ctype=C.c_double):
    return a.ctypes.data_as(C.POINTER(ctype))


def torch_stream():
    """hipStream_t of torch's current stream on the current device (torch owns the stream)."""
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


def make_config(nx, ny, collision="mrt", storage="f32", tau=0.8, lam=3 / 16, eta=1e-7, rho0=1.0,
                u0=(0.0, 0.0), bc=("periodic",) * 4, u_in=(0.0, 0.0), reduce=True, ring=0,
                stream=None):
    cfg = Config()
    cfg.abi_version = ABI_VERSION
    cfg.nx, cfg.ny = int(nx), int(ny)
    cfg.collision = COLLISION.get(collision, collision)
    cfg.storage = STORAGE.get(storage, storage)
    cfg.tau, cfg.lambda_, cfg.eta = float(tau), float(lam), float(eta)
    cfg.rho0, cfg.ux0, cfg.uy0 = float(rho0), float(u0[0]), float(u0[1])
    cfg.bc_xlo, cfg.bc_xhi, cfg.bc_ylo, cfg.bc_yhi = (BC.get(b, b) for b in bc)
    cfg.u_in_x, cfg.u_in_y = float(u_in[0]), float(u_in[1])
    cfg.reduce = 1 if reduce else 0
    cfg.ring = int(ring)
    cfg.stream = stream
    return cfg


def make_body(b):
    """vplbm_body from a dict with the keys of paper_1812_05401_amd.inputs.body."""
    return Body(SHAPE.get(b["kind"], b["kind"]), b["cx"], b["cy"], b.get("r", 0.0), b.get("hx", 0.0),
                b.get("hy", 0.0), b.get("ux", 0.0), b.get("uy", 0.0), b.get("omega", 0.0),
                b.get("ax", 0.0), b.get("ay", 0.0), b.get("freq", 0.0))


# ---- entry points ------------------------------------------------------------------------------

def vplbm_create(cfg):
    h = C.c_void_p()
    check(load().vplbm_create(C.byref(cfg), C.byref(h)))
    return h.value


def vplbm_set_mask(h, body_id, bodies):
    arr = (Body * max(1, len(bodies)))(*[make_body(b) if isinstance(b, dict) else b for b in bodies])
    ids = None
    if body_id is not None:
        body_id = np.ascontiguousarray(body_id, dtype=np.uint8)
        ids = _ptr(body_id, C.c_uint8)
    check(load().vplbm_set_mask(h, ids, arr, len(bodies)))


def vplbm_step(h, n):
    check(load().vplbm_step(h, int(n)))


def vplbm_observables(h, shape=None, fields=False):
    o = Obs()
    rho = ux = uy = None
    ptrs = [None, None, None]
    if fields:
        ny, nx = shape
        rho, ux, uy = (np.empty((ny, nx)) for _ in range(3))
        ptrs = [_ptr(rho), _ptr(ux), _ptr(uy)]
    check(load().vplbm_observables(h, C.byref(o), *ptrs))
    nb = o.nbodies
    obs = {"step": o.step, "mass": o.mass, "fx": np.array(o.fx[:nb]), "fy": np.array(o.fy[:nb]),
           "status": o.status}
    return (obs, rho, ux, uy) if fields else obs


def vplbm_destroy(h):
    check(load().vplbm_destroy(h))


def vplbm_init_fields(h, rho, ux, uy):
    rho, ux, uy = (np.ascontiguousarray(v, dtype=np.float64) for v in (rho, ux, uy))
    check(load().vplbm_init_fields(h, _ptr(rho), _ptr(ux), _ptr(uy)))


def vplbm_get_populations(h, shape):
    ny, nx = shape
    pop = np.empty((9, ny, nx))
    check(load().vplbm_get_populations(h, _ptr(pop)))
    return pop


def vplbm_set_populations(h, pop, step):
    pop = np.ascontiguousarray(pop, dtype=np.float64)
    check(load().vplbm_set_populations(h, _ptr(pop), int(step)))


def vplbm_get_mask(h, shape):
    ids = np.empty(shape, dtype=np.uint8)
    check(load().vplbm_get_mask(h, _ptr(ids, C.c_uint8)))
    return ids


def vplbm_force_series(h, first, count):
    out = np.empty((count, RING_WIDTH))
    check(load().vplbm_force_series(h, int(first), int(count), _ptr(out)))
    return out


def vplbm_momentum_exchange(h, nbodies):
    fx, fy = np.zeros(MAX_BODIES), np.zeros(MAX_BODIES)
    check(load().vplbm_momentum_exchange(h, _ptr(fx), _ptr(fy)))
    return fx[:nbodies], fy[:nbodies]


def vplbm_momentum_exchange_noalloc(h, out_ptr):
    """Momentum exchange into device memory at out_ptr (2 * MAX_BODIES doubles), asynchronously
    on the simulation's stream, without allocating (the library's static scratch)."""
    check(load().vplbm_momentum_exchange_noalloc(h, C.c_void_p(int(out_ptr))))


def vplbm_residual(h):
    r = C.c_double()
    check(load().vplbm_residual(h, C.byref(r)))
    return r.value


def vplbm_steps_per_launch(h):
    n = C.c_int32()
    check(load().vplbm_steps_per_launch(h, C.byref(n)))
    return n.value


def vplbm_steps_done(h):
    n = C.c_int64()
    check(load().vplbm_steps_done(h, C.byref(n)))
    return n.value


def vplbm_stream(h):
    s = C.c_void_p()
    check(load().vplbm_stream(h, C.byref(s)))
    return s.value


def vplbm_bytes_per_update(storage):
    b = C.c_int64()
    check(load().vplbm_bytes_per_update(STORAGE.get(storage, storage), C.byref(b)))
    return b.value


# ---- one handle ---------------------------------------------------------------------------------

class Simulation:
    """A simulation on the GPU.  ``case`` is a paper_1812_05401_amd.inputs.Case (or pass the
    config fields as keywords).  ``stream``: hipStream_t as an int, 'torch' for torch's current
    stream, or None for a stream owned by the library.  ``device_mask``: rasterize the case's
    bodies on the device (True), or leave the lattice all fluid until ``set_mask(body_id,
    bodies)`` gives a host mask (False)."""

    def __init__(self, case=None, stream="torch", reduce=True, ring=0, device_mask=True, **kw):
        if stream == "torch":
            stream = torch_stream()
        if case is not None:
            kw = dict(nx=case.nx, ny=case.ny, collision=case.collision, storage=case.storage,
                      tau=case.tau, lam=case.lam, eta=case.eta, rho0=case.rho0, u0=case.u0,
                      bc=case.bc, u_in=case.u_in, **kw)
        self.cfg = make_config(reduce=reduce, ring=ring, stream=stream, **kw)
        self.nx, self.ny = self.cfg.nx, self.cfg.ny
        self.h = vplbm_create(self.cfg)
        self.nbodies = 0
        if case is not None and case.bodies and device_mask:
            self.set_mask(None, case.bodies)

    @property
    def shape(self):
        return (self.ny, self.nx)

    def set_mask(self, body_id, bodies):
        """body_id: a [ny, nx] uint8 array of body ids (0 = fluid), or None to rasterize
        ``bodies`` on the device."""
        vplbm_set_mask(self.h, body_id, bodies)
        self.nbodies = len(bodies)

    def step(self, n=1):
        vplbm_step(self.h, n)

    def observables(self, fields=False):
        return vplbm_observables(self.h, self.shape, fields)

    def fields(self):
        _, rho, ux, uy = vplbm_observables(self.h, self.shape, True)
        return rho, ux, uy

    def init_fields(self, rho, ux, uy):
        vplbm_init_fields(self.h, rho, ux, uy)

    def populations(self):
        return vplbm_get_populations(self.h, self.shape)

    def set_populations(self, pop, step=0):
        vplbm_set_populations(self.h, pop, step)

    def mask(self):
        return vplbm_get_mask(self.h, self.shape)

    def momentum_exchange(self):
        return vplbm_momentum_exchange(self.h, self.nbodies)

    def residual(self):
        """Relative L2 change of the fluid velocity since the previous call (+inf at the first)."""
        return vplbm_residual(self.h)

    def force_series(self, first, count):
        return vplbm_force_series(self.h, first, count)

    @property
    def steps_done(self):
        return vplbm_steps_done(self.h)

    @property
    def steps_per_launch(self):
        """3 for binary32 storage, else 2 (pairs of steps per launch);
        VPLBM_THREE_STEP=0 caps it at 2 and VPLBM_TWO_STEP=0 at 1."""
        return vplbm_steps_per_launch(self.h)

    @property
    def stream(self):
        return vplbm_stream(self.h)

    def close(self):
        if getattr(self, "h", None):
            vplbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ---- serving pool -----------------------------------------------------------------------------

def _obs_dict(o):
    nb = o.nbodies
    return {"step": o.step, "mass": o.mass, "fx": np.array(o.fx[:nb]), "fy": np.array(o.fy[:nb]),
            "status": o.status}


def case_config(case, **kw):
    return make_config(case.nx, case.ny, collision=case.collision, storage=case.storage,
                       tau=case.tau, lam=case.lam, eta=case.eta, rho0=case.rho0, u0=case.u0,
                       bc=case.bc, u_in=case.u_in, **kw)


def vplbm_pool_bytes_needed(case):
    b = C.c_uint64()
    check(load().vplbm_pool_bytes_needed(C.byref(case_config(case)), C.byref(b)))
    return b.value


class Pool:
    """Continuous-batching pool: ``submit`` queues simulations, ``advance`` retires finished
    ones, admits queued ones within the memory budget and launches the next chunk of steps for
    every resident simulation."""

    def __init__(self, budget_bytes, max_slots=64, steps_per_launch=64, stream=None):
        cfg = PoolConfig(ABI_VERSION, int(budget_bytes), int(max_slots), int(steps_per_launch),
                         stream)
        h = C.c_void_p()
        check(load().vplbm_pool_create(C.byref(cfg), C.byref(h)))
        self.h = h.value
        self.shapes = {}

    def submit(self, case, nsteps=None, keep_fields=False, stop=None):
        """Queue `case` for `nsteps` steps; stop = (tol, every) retires it early once its
        convergence residual over `every` steps is below tol."""
        bodies = case.bodies
        arr = (Body * max(1, len(bodies)))(*[make_body(b) for b in bodies])
        rid = C.c_int64()
        check(load().vplbm_pool_submit(self.h, C.byref(case_config(case)), arr, len(bodies),
                                       int(nsteps if nsteps is not None else case.steps),
                                       1 if keep_fields else 0, C.byref(rid)))
        self.shapes[rid.value] = (case.ny, case.nx)
        if stop is not None:
            check(load().vplbm_pool_set_stop(self.h, rid.value, float(stop[0]), int(stop[1])))
        return rid.value

    def cancel(self, rid):
        check(load().vplbm_pool_cancel(self.h, int(rid)))

    def set_admission(self, max_resident_nodes):
        """Cap on the resident lattice nodes (0: none)."""
        check(load().vplbm_pool_set_admission(self.h, int(max_resident_nodes)))

    def residual(self, rid):
        r = C.c_double()
        check(load().vplbm_pool_residual(self.h, int(rid), C.byref(r)))
        return r.value

    def advance(self):
        r, q, f = C.c_int32(), C.c_int32(), C.c_int32()
        check(load().vplbm_pool_advance(self.h, C.byref(r), C.byref(q), C.byref(f)))
        return r.value, q.value, f.value

    def status(self, rid):
        st, n = C.c_int32(), C.c_int64()
        check(load().vplbm_pool_status(self.h, int(rid), C.byref(st), C.byref(n)))
        return st.value, n.value

    def result(self, rid, fields=False):
        o = Obs()
        ptrs = [None, None, None]
        out = None
        if fields:
            out = tuple(np.empty(self.shapes[rid]) for _ in range(3))
            ptrs = [_ptr(a) for a in out]
        check(load().vplbm_pool_result(self.h, int(rid), C.byref(o), *ptrs))
        self.shapes.pop(rid, None)
        return (_obs_dict(o), out) if fields else _obs_dict(o)

    def close(self):
        if getattr(self, "h", None):
            check(load().vplbm_pool_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
