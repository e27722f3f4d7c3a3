"""Two and three steps per launch (the intermediate steps kept in LDS) against one step per
launch.  The populations must be bitwise the same in every storage format and edge combination,
over graph replays, odd remainders and restarts.  The per-step ring values (mass, body forces) are
FP64 sums over different tilings, so they agree up to summation order (1e-13 relative).  Three
steps per launch exist for binary32 storage (the convective outlet included); elsewhere a request
for them gets two."""
import contextlib
import os

import numpy as np
import pytest

from paper_1812_05401_amd import inputs as I
from tests.helpers import gpu_sim
from tests.test_gpu_parity import CASES, build_case

pytestmark = pytest.mark.gpu

STORAGES = ["f64", "f32", "f32d", "f16s", "bf16s", "f16sr", "bf16sr"]
# every parity case takes the two-step kernel: static, spinning and moving bodies, host masks,
# every edge combination and the convective outlet
TWO = CASES


@contextlib.contextmanager
def env(**kw):
    old = {k: os.environ.get(k) for k in kw}
    os.environ.update({k: str(v) for k, v in kw.items()})
    try:
        yield
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def expected_spl(case, storage, spl):
    """Steps per launch the library takes when asked for at most spl (True: 2, False: 1)."""
    spl = int(spl) + 1 if isinstance(spl, bool) else spl
    if spl == 3 and storage != "f32":
        return 2
    return spl


def make(case, ids, storage, fields, spl, capfd=None, graph_steps=None):
    """A GPU simulation with at most spl steps per launch (True: two, False: one)."""
    spl = int(spl) + 1 if isinstance(spl, bool) else spl
    extra = {} if graph_steps is None else {"VPLBM_GRAPH_STEPS": graph_steps}
    with env(VPLBM_TWO_STEP=int(spl >= 2), VPLBM_THREE_STEP=int(spl >= 3), VPLBM_LOG=1, **extra):
        s = gpu_sim(case, storage=storage, device_mask=ids is None)
        if ids is not None:
            s.set_mask(ids, case.bodies)
    want = expected_spl(case, storage, spl)
    if capfd is not None:
        assert last_report(capfd) == want
    assert s.steps_per_launch == want
    s.init_fields(*fields)
    return s


def last_report(capfd):
    """The last 'steps per launch' figure the library logged (at create or set_mask)."""
    err = capfd.readouterr().err
    flags = [int(l.rsplit(" ", 1)[1]) for l in err.splitlines() if "steps per launch" in l]
    assert flags, err[-400:]
    return flags[-1]


def same_run(a, b, first, count, what):
    pa, pb = a.populations(), b.populations()
    assert np.array_equal(pa, pb), f"{what}: populations differ at {np.argwhere(pa != pb)[:3]}"
    sa, sb = a.force_series(first, count), b.force_series(first, count)
    scale = np.maximum(np.max(np.abs(sb), axis=0), 1e-300)
    d = np.max(np.abs(sa - sb) / scale)
    assert d <= 1e-13, f"{what}: ring values differ by {d:.2e}"
    oa, ob = a.observables(), b.observables()
    assert oa["step"] == ob["step"] and oa["status"] == ob["status"] == 0


@pytest.mark.parametrize("storage", STORAGES)
@pytest.mark.parametrize("spec", TWO, ids=[c[0] for c in TWO])
def test_two_step_bitwise_equals_one_step(gpu, capfd, spec, storage):
    """101 steps (three 32-step graph replays, two two-step launches and a one-step launch), then
    1 and 3 more: bitwise the same populations as one step per launch."""
    case, ids = build_case(*spec, seed=11)
    fields = I.random_fields(case.nx, case.ny, 11, u_mean=case.u_in)
    a = make(case, ids, storage, fields, True, capfd, graph_steps=32)
    b = make(case, ids, storage, fields, False, capfd, graph_steps=32)
    done = 0
    for n in (101, 1, 3):
        a.step(n)
        b.step(n)
        done += n
        same_run(a, b, 0, done, f"{spec[0]}/{storage} after {done} steps")
    a.close()
    b.close()


@pytest.mark.parametrize("spec", TWO, ids=[c[0] for c in TWO])
def test_three_step_bitwise_equals_one_step(gpu, capfd, spec):
    """Binary32 storage with three steps per launch (the convective outlet included): 101 steps
    (three 32-step graph replays of ten three-step launches and a two-step one each, then a
    three-step and a two-step launch), then 1, 3, 2 and 5 more: bitwise the same populations as
    one step per launch."""
    case, ids = build_case(*spec, seed=12)
    fields = I.random_fields(case.nx, case.ny, 12, u_mean=case.u_in)
    a = make(case, ids, "f32", fields, 3, capfd, graph_steps=32)
    b = make(case, ids, "f32", fields, False, capfd, graph_steps=32)
    done = 0
    for n in (101, 1, 3, 2, 5):
        a.step(n)
        b.step(n)
        done += n
        same_run(a, b, 0, done, f"{spec[0]}/f32 three steps per launch after {done} steps")
    a.close()
    b.close()


@pytest.mark.parametrize("storage,spl", [("f64", 2), ("f32", 3)])
def test_two_step_ring_and_restart(gpu, storage, spl):
    """Mixed call sizes with observations in between (each observation folds the last steps),
    then a restart from populations at an odd step: ring entries and populations match the
    one-step path."""
    spec = CASES[2]                                           # channel with two disks
    case, ids = build_case(*spec, seed=21)
    fields = I.random_fields(case.nx, case.ny, 21, u_mean=case.u_in)
    a = make(case, ids, storage, fields, spl, graph_steps=32)
    b = make(case, ids, storage, fields, False, graph_steps=32)
    done = 0
    for n in (2, 1, 2, 64, 5, 33, 4, 3, 7):
        a.step(n)
        b.step(n)
        done += n
        assert a.observables()["mass"] == pytest.approx(b.observables()["mass"], rel=1e-14)
    same_run(a, b, 0, done, "mixed calls")
    pop = b.populations()
    t0 = 1001
    a.set_populations(pop, t0)
    b.set_populations(pop, t0)
    a.step(37)
    b.step(37)
    same_run(a, b, t0, 37, "after a restart at an odd step")
    a.close()
    b.close()


@pytest.mark.parametrize("nx,ny,storage,steps", [
    (2048, 512, "f32", 200),
    (8192, 2048, "f16s", 130),
    (8192, 2048, "f32", 130),
    (2100, 2001, "bf16sr", 21),
    (6048, 2016, "f32", 131),
    (2048, 512, "f32", 20000),
    (2048, 512, "f16sr", 20000),
], ids=["wake_2048x512_f32", "wake_8192x2048_f16s", "wake_8192x2048_f32", "ragged_tall_tiles_bf16sr",
        "paper_re500_convective_f32", "wake_2048x512_f32_20k_steps", "wake_2048x512_f16sr_20k_steps"])
def test_two_step_full_size(gpu, nx, ny, storage, steps):
    """The benchmark lattices in the launch configuration the benchmark times (graph replays of
    three-step launches for binary32, two-step launches otherwise, non-temporal stores on the large
    lattice), a ragged lattice large enough for the tall 2-byte tiles, and the paper's Re = 500
    cylinder with its convective outlet (three steps per launch)."""
    if (nx, ny) == (6048, 2016):
        case = I.paper_cylinder_re500(storage=storage)
    else:
        case = I.cylinder_wake(nx, ny, storage=storage)
    assert (case.nx, case.ny) == (nx, ny)
    fields = I.random_fields(case.nx, case.ny, 4, u_mean=case.u_in)
    a = make(case, None, storage, fields, 3)
    b = make(case, None, storage, fields, False)
    a.step(steps)
    b.step(steps)
    first = max(0, steps - 4096)                  # the ring holds the last 4096 steps
    same_run(a, b, first, steps - first, f"{case.name}/{storage}, {steps} steps")
    a.close()
    b.close()


@pytest.mark.parametrize("spl", [2, 3])
def test_two_step_oscillating_cylinder_full_size(gpu, spl):
    """The 8192 x 2048 oscillating cylinder (mask rebuilt on the device every step, swept box
    only): two or three steps per launch with each step's own mask, bitwise the one-step run."""
    case = I.oscillating_cylinder_8192x2048()
    fields = I.random_fields(case.nx, case.ny, 6, u_mean=case.u_in)
    a = make(case, None, "f32", fields, spl)
    b = make(case, None, "f32", fields, False)
    for n in (2, 37, 64):
        a.step(n)
        b.step(n)
    same_run(a, b, 0, 103, "oscillating_cylinder_8192x2048")
    assert np.array_equal(a.mask(), b.mask())
    a.close()
    b.close()


@pytest.mark.parametrize("spl", [2, 3])
def test_two_step_without_reductions_and_with_a_short_ring(gpu, spl):
    """Reductions off: the populations are those of the reduced run, bitwise.  A ring of 16 steps
    over 101 steps (the folds wrap around it): its last 16 entries match one step per launch."""
    spec = CASES[2]
    case, ids = build_case(*spec, seed=31)
    fields = I.random_fields(case.nx, case.ny, 31, u_mean=case.u_in)
    with env(VPLBM_TWO_STEP=1, VPLBM_THREE_STEP=int(spl == 3)):
        a = gpu_sim(case, storage="f32", reduce=False)
        b = gpu_sim(case, storage="f32", ring=16)
    with env(VPLBM_TWO_STEP=0):
        c = gpu_sim(case, storage="f32", ring=16)
    for s in (a, b, c):
        s.init_fields(*fields)
        s.step(101)
    assert a.steps_per_launch == spl and b.steps_per_launch == spl and c.steps_per_launch == 1
    assert np.array_equal(a.populations(), b.populations())
    same_run(b, c, 85, 16, "ring of 16")
    for s in (a, b, c):
        s.close()


@pytest.mark.parametrize("spl", [2, 3])
def test_bodies_start_moving_mid_run(gpu, spl):
    """Static bodies for 33 steps, then the same bodies set oscillating (the extra masks are
    allocated then, after the graphs were captured), 65 more: bitwise the one-step path."""
    case = I.cylinder_wake(300, 120, d=20.0, x0=80.0, re=100.0, storage="f32")
    moving = [dict(b, ax=0.0, ay=4.0, freq=0.01) for b in case.bodies]
    fields = I.random_fields(case.nx, case.ny, 8, u_mean=case.u_in)
    a = make(case, None, "f32", fields, spl, graph_steps=32)
    b = make(case, None, "f32", fields, False, graph_steps=32)
    for s in (a, b):
        s.step(33)
        with env(VPLBM_THREE_STEP=int(spl == 3)):
            s.set_mask(None, moving)
        s.step(65)
    assert a.steps_per_launch == spl and b.steps_per_launch == 1
    same_run(a, b, 0, 98, "bodies start moving")
    assert np.array_equal(a.mask(), b.mask())
    a.close()
    b.close()


@pytest.mark.parametrize("spl,seed", [(2, 2024), (3, 3033)])
def test_two_step_random_configurations(gpu, spl, seed):
    """24 seeded random configurations: lattice sizes from 2 x 1 to 300 x 200, every edge
    combination (periodic, channel, periodic in x with free-slip walls, convective outlet),
    0-3 bodies (static, spinning or oscillating), every storage format (binary32 every other
    configuration when three steps per launch are asked for) and 1-41 steps; the populations and
    ring values of two or three steps per launch against one step per launch."""
    from paper_1812_05401_amd import binding as B
    rng = np.random.default_rng(seed)
    pfs = (I.PERIODIC, I.PERIODIC, I.FREESLIP, I.FREESLIP)
    bcs = [I.ALL_PERIODIC, I.CHANNEL, pfs, I.CHANNEL_CONVECTIVE]
    done = 0
    for k in range(24):
        nx, ny = int(rng.integers(2, 301)), int(rng.integers(1, 201))
        bc = bcs[int(rng.integers(len(bcs)))]
        storage = STORAGES[int(rng.integers(len(STORAGES)))]
        if spl == 3 and k % 2 == 0:
            storage = "f32"
        nb = int(rng.integers(0, 4)) if min(nx, ny) >= 12 else 0
        moving = bool(rng.random() < 0.4)
        bodies = I.random_bodies(nx, ny, 100 + k, nb, moving=moving, rmin=1.5,
                                 rmax=max(2.0, min(nx, ny) / 5)) if nb else []
        u_in = (0.04, 0.0) if bc[0] == I.VELOCITY else (0.0, 0.0)
        case = I.Case(f"random{k}", nx, ny, collision="mrt" if k % 2 else "srt",
                      tau=float(rng.uniform(0.55, 1.2)), lam=3 / 16, bc=bc, u_in=u_in, u0=u_in,
                      bodies=bodies, storage=storage)
        fields = I.random_fields(nx, ny, 200 + k, u_mean=u_in)
        steps = int(rng.integers(1, 42))
        try:
            a = make(case, None, storage, fields, spl)
        except B.VplbmError as e:              # a lattice the edge rules do not admit
            assert e.code == B.EINVAL, e
            continue
        b = make(case, None, storage, fields, False)
        a.step(steps)
        b.step(steps)
        same_run(a, b, 0, steps, f"{case.name} {nx}x{ny} {bc} {storage} {len(bodies)} bodies, {steps} steps")
        a.close()
        b.close()
        done += 1
    assert done >= 20
