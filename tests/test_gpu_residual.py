"""Convergence residual on the GPU (the relative L2 change of the fluid velocity, Eq. 20 with the
earlier field as the reference): vplbm_residual against the oracle's, and the serving pool's
early stop of steady runs against the single-simulation path."""
import math
import zlib

import numpy as np
import pytest

from paper_1812_05401_amd import inputs as I
from paper_1812_05401_amd import sweeps as S
from tests.helpers import rel_err
from tests.test_gpu_parity import CASES, build_case, make_pair

pytestmark = pytest.mark.gpu

RES_CASES = [CASES[i] for i in (0, 2, 5, 13)]


@pytest.mark.parametrize("spec", RES_CASES, ids=[c[0] for c in RES_CASES])
def test_residual_matches_oracle(gpu, spec):
    """Two successive residuals after 150 + 100 + 50 steps.  r is a ratio of FP64 sums; the
    fields agree to 1e-12 of their maximum, so r agrees to about 1e-12 times max|u| / rms|u|."""
    seed = zlib.crc32(spec[0].encode()) % 10000
    case, ids = build_case(*spec, seed=seed)
    o, g = make_pair(case, ids, seed)
    o.step(150)
    g.step(150)
    assert math.isinf(g.residual())
    for n in (100, 50):
        _, ux0, uy0 = o.fields()
        o.step(n)
        g.step(n)
        r_o = o.residual(ux0, uy0)
        r_g = g.residual()
        print(f"{spec[0]}: residual over {n} steps {r_o:.6e}, GPU - oracle {r_g - r_o:.2e}", flush=True)
        assert r_o > 1e-5
        assert abs(r_g - r_o) <= 1e-11


def _drain(pool, ids):
    from paper_1812_05401_amd import binding as B
    out = {}
    while len(out) < len(ids):
        pool.advance()
        for rid in ids:
            if rid in out:
                continue
            st, done = pool.status(rid)
            if st in (B.DONE, B.FAILED):
                res = pool.residual(rid)
                out[rid] = (st, done, res) + pool.result(rid, fields=True)
    return out


@pytest.mark.parametrize("spl,every,storage,tol", [(64, 256, "f64", 1e-6), (7, 280, "f64", 1e-6),
                                                   (64, 256, "f32", 1e-5), (7, 280, "f32", 1e-5)])
def test_pool_early_stop(gpu, spl, every, storage, tol):
    """A steady plane-shear run with an early stop retires at the first check whose residual is
    below the tolerance, one step after it; its result is the single-simulation run of as many
    steps.  A run whose tolerance is never met runs all its steps, and a run without a stop is
    not affected.  With an odd steps_per_launch the final step after the stop is the single step
    of a replay's first launch.  Binary32 runs take three steps per launch on 14-row tiles."""
    B = gpu
    steady = S.shear_case("srt", 0.5 + math.sqrt(6) / 4).case
    never = S.shear_case("mrt", 1.5, 3 / 16, nx=32).case
    plain = I.Case("plain", 90, 60, collision="mrt", tau=0.7, bc=I.CHANNEL, u_in=(0.04, 0.0),
                   u0=(0.04, 0.0), bodies=[I.body("disk", 30, 29.5, r=6)], storage="f64")
    for c in (steady, never, plain):
        c.storage = storage
    pool = B.Pool(1 << 30, max_slots=4, steps_per_launch=spl)
    a = pool.submit(steady, 400_000, keep_fields=True, stop=(tol, every))
    b = pool.submit(never, 3 * every, keep_fields=True, stop=(1e-300, every))
    c = pool.submit(plain, 1000, keep_fields=True)
    res = _drain(pool, [a, b, c])
    pool.close()

    st, done, r, obs, (rho, ux, uy) = res[a]
    assert st == B.DONE and done < 400_000
    check = done - 1
    assert check % every == 0 and check >= 3 * every
    assert r < tol and obs["step"] == done - 1
    print(f"steady shear stopped after {done} steps, residual {r:.3e}", flush=True)
    s = B.Simulation(steady, stream=None)
    s.step(check - 2 * every)
    s.residual()
    s.step(every)
    r_prev = s.residual()
    s.step(every)
    r_single = s.residual()
    s.step(1)
    so, srho, sux, suy = s.observables(fields=True)
    s.close()
    assert r_prev >= tol                                   # the stop came at the first chance
    assert abs(r_single - r) <= 1e-9 * r
    assert rel_err(rho, srho) <= 1e-13 and rel_err(np.stack([ux, uy]), np.stack([sux, suy])) <= 1e-12
    assert abs(obs["mass"] - so["mass"]) <= 1e-13 * so["mass"]

    st, done, r, obs, _ = res[b]
    assert st == B.DONE and done == 3 * every and 0 < r < math.inf

    st, done, r, obs, (rho, ux, uy) = res[c]
    assert st == B.DONE and done == 1000 and math.isinf(r)
    s = B.Simulation(plain, stream=None)
    s.step(1000)
    _, srho, sux, suy = s.observables(fields=True)
    s.close()
    assert rel_err(np.stack([ux, uy]), np.stack([sux, suy])) <= 1e-12


def test_pool_stop_arguments(gpu):
    B = gpu
    pool = B.Pool(1 << 30, max_slots=2, steps_per_launch=8)
    case = S.shear_case("srt", 0.8, steps=100).case
    rid = pool.submit(case)
    for tol, every in ((0.0, 10), (-1.0, 10), (float("nan"), 10), (1e-6, 0)):
        with pytest.raises(B.VplbmError) as e:
            B.check(B.load().vplbm_pool_set_stop(pool.h, rid, tol, every))
        assert e.value.code == B.EINVAL
    need = B.vplbm_pool_bytes_needed(case)
    small = B.Pool(need, max_slots=1, steps_per_launch=8)
    with pytest.raises(B.VplbmError) as e:
        small.submit(case, stop=(1e-6, 10))                # the snapshot does not fit the budget
    assert e.value.code == B.EBUDGET
    small.close()
    pool.advance()                                         # admitted: too late for a stop
    with pytest.raises(B.VplbmError) as e:
        B.check(B.load().vplbm_pool_set_stop(pool.h, rid, 1e-6, 10))
    assert e.value.code == B.ESTATE
    pool.close()


def test_pool_early_stop_with_convective_outlet(gpu):
    """A steady low-Reynolds channel flow past a disk with the convective outlet stops at the
    first check below the tolerance; the pool's residual (which reads the outlet's recorded
    values) and fields are those of the single-simulation run."""
    B = gpu
    tol, every = 1e-7, 256                      # checks fall on graph-replay boundaries (64 steps)
    case = I.Case("conv_steady", 90, 60, collision="mrt", tau=0.7, bc=I.CHANNEL_CONVECTIVE,
                  u_in=(0.04, 0.0), u0=(0.04, 0.0), bodies=[I.body("disk", 30, 29.5, r=6)],
                  storage="f64")
    pool = B.Pool(1 << 30, max_slots=2, steps_per_launch=64)
    a = pool.submit(case, 400_000, keep_fields=True, stop=(tol, every))
    st, done, r, obs, (rho, ux, uy) = _drain(pool, [a])[a]
    pool.close()
    assert st == B.DONE and done < 400_000
    check = done - 1
    assert check % every == 0 and check >= 3 * every and r < tol
    print(f"convective channel stopped after {done} steps, residual {r:.3e}", flush=True)
    s = B.Simulation(case, stream=None)
    s.step(check - 2 * every)
    s.residual()
    s.step(every)
    r_prev = s.residual()
    s.step(every)
    r_single = s.residual()
    s.step(1)
    so, srho, sux, suy = s.observables(fields=True)
    s.close()
    assert r_prev >= tol
    assert abs(r_single - r) <= 1e-9 * r
    assert np.array_equal(rho, srho) and np.array_equal(ux, sux) and np.array_equal(uy, suy)
