"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on the same seeded
inputs.  FP64 storage must agree to 1e-12 relative after 1000 steps on populations, density,
velocity, mass and body forces; masks must agree exactly."""
import zlib

import numpy as np
import pytest

from paper_1812_05401_amd import inputs as I
from tests.helpers import couette_l2, force_scale, gpu_sim, host_threads, oracle_sim, rel_err

pytestmark = pytest.mark.gpu

TOL64 = 1e-12

P4 = I.ALL_PERIODIC
CH = I.CHANNEL
PFS = (I.PERIODIC, I.PERIODIC, I.FREESLIP, I.FREESLIP)

# name, nx, ny, collision, tau, lam, eta, bc, u_in, nbodies, moving, host_mask
CASES = [
    ("periodic_srt", 131, 67, "srt", 0.7, 3 / 16, 1e-7, P4, (0.0, 0.0), 3, False, False),
    ("periodic_mrt", 131, 67, "mrt", 0.6, 3 / 16, 1e-7, P4, (0.0, 0.0), 3, False, False),
    ("channel_mrt", 200, 45, "mrt", 0.56, 3 / 16, 1e-7, CH, (0.05, 0.0), 2, False, False),
    ("channel_srt_uy", 200, 45, "srt", 0.58, 3 / 16, 1e-7, CH, (0.04, 0.005), 2, False, False),
    ("freeslip_mrt_eta1", 97, 50, "mrt", 0.9, 3 / 8, 1.0, PFS, (0.0, 0.0), 2, False, False),
    ("moving_mrt", 160, 70, "mrt", 0.6, 3 / 16, 1e-7, CH, (0.05, 0.0), 2, True, False),
    ("moving_srt_periodic", 90, 75, "srt", 0.75, 3 / 16, 1e-7, P4, (0.0, 0.0), 3, True, False),
    ("hostmask_srt_channel", 70, 33, "srt", 0.8, 3 / 16, 1e-7, CH, (0.03, 0.0), 3, False, True),
    ("hostmask_mrt_channel", 70, 33, "mrt", 0.65, 3 / 16, 1e-3, CH, (0.03, 0.0), 4, False, True),
    ("tiny_periodic", 3, 3, "mrt", 0.7, 3 / 16, 1e-7, P4, (0.0, 0.0), 0, False, False),
    ("tiny_channel", 5, 4, "srt", 0.7, 3 / 16, 1e-7, CH, (0.03, 0.0), 0, False, False),
    ("wide_ragged", 517, 9, "mrt", 0.7, 3 / 16, 1e-7, PFS, (0.0, 0.0), 2, False, False),
    ("tall_ragged", 65, 300, "srt", 0.9, 3 / 16, 1e-7, CH, (0.05, 0.0), 2, False, False),
    ("convective_srt", 150, 40, "srt", 0.56, 3 / 16, 1e-7, I.CHANNEL_CONVECTIVE, (0.05, 0.0), 2, False, False),
    ("convective_mrt_moving", 150, 40, "mrt", 0.6, 3 / 16, 1e-7, I.CHANNEL_CONVECTIVE, (0.04, 0.0), 2, True, False),
]


def build_case(name, nx, ny, coll, tau, lam, eta, bc, u_in, nb, moving, host_mask, seed,
               storage="f64"):
    bodies = I.random_bodies(nx, ny, seed, nb, moving=moving, rmin=1.5,
                             rmax=max(2.0, min(nx, ny) / 5)) if nb else []
    case = I.Case(name, nx, ny, collision=coll, storage=storage, tau=tau, lam=lam, eta=eta,
                  bc=bc, u_in=u_in, bodies=bodies, u0=u_in)
    ids = None
    if host_mask:
        # a random porous medium: scattered solid nodes of bodies at rest
        for b in bodies:
            b.update(ux=0.0, uy=0.0, omega=0.0)
        r = np.random.default_rng(seed + 1000)
        ids = np.where(r.random((ny, nx)) < 0.25, r.integers(1, nb + 1, (ny, nx)), 0).astype(np.uint8)
    return case, ids


def make_pair(case, ids, seed, storage="f64"):
    fields = I.random_fields(case.nx, case.ny, seed, u_mean=case.u_in)
    o = oracle_sim(case, rasterize=ids is None, init=False)
    if ids is not None:
        o.set_mask(ids)
    o.init_fields(*fields)
    g = gpu_sim(case, storage=storage, device_mask=ids is None)
    if ids is not None:
        g.set_mask(ids, case.bodies)
    g.init_fields(*fields)
    return o, g


def compare(o, g, tol, what=""):
    assert np.array_equal(g.mask(), o.mask()), f"{what}: masks differ"
    eg = rel_err(g.populations(), o.populations())
    ob_o = o.obs()
    ob_g = g.observables()
    assert ob_g["status"] == 0
    assert ob_g["step"] == ob_o["step"]
    em = abs(ob_g["mass"] - ob_o["mass"]) / abs(ob_o["mass"])
    ef = 0.0
    if len(ob_o["fx"]):
        sc = force_scale(ob_o)
        ef = max(np.max(np.abs(ob_g["fx"] - ob_o["fx"])), np.max(np.abs(ob_g["fy"] - ob_o["fy"]))) / sc
    rho_o, ux_o, uy_o = o.fields()
    rho_g, ux_g, uy_g = g.fields()
    er = rel_err(rho_g, rho_o)
    eu = rel_err(np.stack([ux_g, uy_g]), np.stack([ux_o, uy_o]))
    print(f"{what}: pop {eg:.2e} rho {er:.2e} u {eu:.2e} mass {em:.2e} force {ef:.2e}", flush=True)
    return eg, er, eu, em, ef


@pytest.mark.parametrize("spec", CASES, ids=[c[0] for c in CASES])
def test_fp64_parity_1000_steps(gpu, spec):
    seed = zlib.crc32(spec[0].encode()) % 10000
    case, ids = build_case(*spec, seed=seed)
    o, g = make_pair(case, ids, seed)
    assert np.array_equal(g.mask(), o.mask())
    o.step(1000)
    g.step(1000)
    errs = compare(o, g, TOL64, spec[0])
    assert max(errs) <= TOL64


def test_taylor_couette_128_parity(gpu):
    """The 128 x 128 FP64 SRT Taylor-Couette case from its uniform start, 1000 steps."""
    case = I.taylor_couette_128()
    o = oracle_sim(case)
    g = gpu_sim(case)
    assert np.array_equal(g.mask(), o.mask())
    assert rel_err(g.populations(), o.populations()) <= 1e-15
    o.step(1000)
    g.step(1000)
    assert max(compare(o, g, TOL64, "taylor_couette_128")) <= TOL64


def test_graph_replay_equals_single_steps(gpu):
    """Chunks replayed from the captured graph run the same kernels as one-step launches."""
    case, _ = build_case(*CASES[2], seed=5)
    fields = I.random_fields(case.nx, case.ny, 5, u_mean=case.u_in)
    a = gpu_sim(case)
    b = gpu_sim(case)
    a.init_fields(*fields)
    b.init_fields(*fields)
    a.step(300)                                   # two 128-step graph replays and 44 launches
    for _ in range(300):
        b.step(1)
    assert np.array_equal(a.populations(), b.populations())
    oa, ob = a.observables(), b.observables()
    assert oa["step"] == ob["step"] == 299
    assert abs(oa["mass"] - ob["mass"]) <= 1e-13 * abs(ob["mass"])


def test_force_series_matches_oracle_every_step(gpu):
    case, _ = build_case(*CASES[5], seed=9)
    o, g = make_pair(case, None, 9)
    want = []
    for _ in range(70):
        o.step(1)
        ob = o.obs()
        want.append((ob["mass"], ob["fx"], ob["fy"], force_scale(ob)))
    g.step(70)
    ser = g.force_series(0, 70)
    for t, (m, fx, fy, sc) in enumerate(want):
        assert abs(ser[t, 0] - m) <= TOL64 * m
        nb = len(fx)
        assert np.max(np.abs(ser[t, 1:1 + 2 * nb:2] - fx)) <= TOL64 * sc
        assert np.max(np.abs(ser[t, 2:2 + 2 * nb:2] - fy)) <= TOL64 * sc


@pytest.mark.parametrize("storage", ["f64", "f32", "f32d", "f16s", "bf16s"])
def test_checkpoint_resume_is_bitwise(gpu, storage):
    """A checkpoint (populations decoded to FP64) restores the stored bits in every format, so a
    resumed run continues bit for bit (binary32 deviations below 2^-33, which could come back
    changed, do not occur in this state)."""
    case, _ = build_case(*CASES[0], seed=3, storage=storage)
    fields = I.random_fields(case.nx, case.ny, 3)
    a = gpu_sim(case)
    a.init_fields(*fields)
    a.step(300)
    pop = a.populations()
    a.step(300)
    b = gpu_sim(case)
    b.set_populations(pop, 300)
    assert np.array_equal(b.populations(), pop)
    b.step(300)
    assert b.steps_done == 600
    assert np.array_equal(a.populations(), b.populations())


def test_unstable_state_is_reported(gpu):
    """A non-finite velocity or a non-positive density (forced from the host through the
    initial fields) sets the status word; the next step call is refused."""
    from paper_1812_05401_amd import binding as B
    case, _ = build_case(*CASES[9], seed=1)
    zeros = np.zeros((3, 3))
    bad_u = zeros.copy()
    bad_u[1, 1] = np.nan
    for rho, ux in ((np.ones((3, 3)), bad_u), (-np.ones((3, 3)), zeros)):
        g = gpu_sim(case)
        g.init_fields(rho, ux, zeros)
        g.step(2)
        assert g.observables()["status"] == 1
        with pytest.raises(B.VplbmError) as e:
            g.step(1)
        assert e.value.code == B.EUNSTABLE
        g.close()


def test_full_size_cylinder_2048x512(gpu):
    """The 2048 x 512 cylinder wake at its full size, in FP64 and in the FP32 the benchmark
    times, from the uniform start: FP32 after 40 steps (single launches), FP64 after 130 (one
    128-step graph replay, then a two-step launch)."""
    case = I.cylinder_wake_2048x512()
    o = oracle_sim(case)
    o.step(40)
    g32 = gpu_sim(case, storage="f32")
    g32.step(40)
    eg, er, eu, em, ef = compare(o, g32, 0, "cylinder_2048x512_f32")
    # FP32: a few roundings of ~6e-8 per step on populations of size <= 0.45
    assert eg < 1e-5 and er < 1e-5 and eu < 1e-4 and em < 1e-6 and ef < 1e-4
    g32.close()
    o.step(90)
    g64 = gpu_sim(case, storage="f64")
    g64.step(130)
    assert max(compare(o, g64, TOL64, "cylinder_2048x512_f64")) <= TOL64


def test_full_size_cylinder_2048x512_fp64_1000_steps(gpu):
    """The 2048 x 512 cylinder wake at its full size, FP64 storage, after 1000 steps from the
    uniform start (seven 128-step graph replays of two-step launches, then direct launches), in
    the launch configuration the benchmark times for this lattice: populations, fields, mass and
    force to 1e-12 relative of the oracle (run on the host's threads; its results do not depend
    on their number)."""
    case = I.cylinder_wake_2048x512()
    o = oracle_sim(case, threads=host_threads())
    o.step(1000)
    g = gpu_sim(case, storage="f64")
    assert g.steps_per_launch == 2
    g.step(1000)
    assert max(compare(o, g, TOL64, "cylinder_2048x512_f64_1000")) <= TOL64


def test_taylor_couette_128_eq21_on_the_gpu(gpu):
    """The 128 x 128 Taylor-Couette case over its whole 5000 steps on the GPU (FP64): the relative
    L2 error of the velocity against the analytic profile (Eq. 21 through Eq. 20) is the oracle's
    to 1e-9 of itself, about 2.7% (the staircase walls), and the fields match to 1e-12."""
    case = I.taylor_couette_128()
    o = oracle_sim(case, threads=host_threads())
    o.step(case.steps)
    g = gpu_sim(case)
    g.step(case.steps)
    assert max(compare(o, g, TOL64, "taylor_couette_128_5000")) <= TOL64
    R1, R2 = case.bodies[0]["r"], case.bodies[1]["r"]
    ud = case.bodies[0]["omega"] * R1
    _, ux_o, uy_o = o.fields()
    _, ux_g, uy_g = g.fields()
    e_o = couette_l2(ux_o, uy_o, o.mask(), case.nx, R1, R2, ud)
    e_g = couette_l2(ux_g, uy_g, g.mask(), case.nx, R1, R2, ud)
    print(f"taylor_couette_128: L2 vs Eq. 21 GPU {e_g[0]:.6e} (v {e_g[1]:.6e}), "
          f"oracle {e_o[0]:.6e} (v {e_o[1]:.6e})", flush=True)
    assert 0.02 < e_g[0] < 0.03
    for a, b in zip(e_g, e_o):
        assert abs(a - b) <= 1e-9 * b


def test_full_size_paper_cylinder_re500(gpu):
    """The paper's 6048 x 2016 Re = 500 case (SRT, convective outlet) at its full size, 3 steps
    from the uniform start, FP64 and FP32 storage against the oracle."""
    case = I.paper_cylinder_re500()
    o = oracle_sim(case)
    o.step(3)
    g64 = gpu_sim(case, storage="f64")
    g64.step(3)
    assert max(compare(o, g64, TOL64, "paper_cylinder_f64")) <= TOL64
    g64.close()
    g32 = gpu_sim(case, storage="f32")
    g32.step(3)
    eg, er, eu, em, ef = compare(o, g32, 0, "paper_cylinder_f32")
    assert eg < 1e-5 and er < 1e-5 and eu < 1e-4 and em < 1e-6 and ef < 1e-4


def test_full_size_oscillating_cylinder_8192x2048(gpu):
    """The 8192 x 2048 oscillating cylinder at its full size in the launch configuration the
    benchmark times (non-temporal stores, mask rebuilt on the device every step), 3 steps from the
    uniform start: FP64 against the oracle to 1e-12, FP32 and FP16S to their rounding."""
    case = I.oscillating_cylinder_8192x2048()
    o = oracle_sim(case)
    o.step(3)
    for storage, tol in (("f64", None), ("f32", (1e-5, 1e-4)), ("f16s", (2e-3, 2e-2))):
        g = gpu_sim(case, storage=storage)
        g.step(3)
        errs = compare(o, g, TOL64 if tol is None else 0, f"oscillating_8192x2048_{storage}")
        g.close()
        if tol is None:
            assert max(errs) <= TOL64
        else:
            eg, er, eu, em, ef = errs
            assert eg < tol[0] and er < tol[0] and eu < tol[1] and em < tol[0] and ef < tol[1]


ME_CASES = [CASES[i] for i in (0, 2, 5, 13)]


@pytest.mark.parametrize("spec", ME_CASES, ids=[c[0] for c in ME_CASES])
def test_momentum_exchange_matches_oracle(gpu, spec):
    """The link-based force over the post-collision state after 200 steps.  Scale: the summed
    magnitude of the link terms, bounded by (number of fluid-solid links) x 2 max f."""
    seed = zlib.crc32(spec[0].encode()) % 10000
    case, ids = build_case(*spec, seed=seed)
    o, g = make_pair(case, ids, seed)
    o.step(200)
    g.step(200)
    ofx, ofy = o.momentum_exchange()
    gfx, gfy = g.momentum_exchange()
    solid = o.mask() != 0
    links = sum(int(np.sum(~solid & np.roll(solid, (-ey, -ex), axis=(0, 1))))
                for ex in (-1, 0, 1) for ey in (-1, 0, 1) if ex or ey)
    sc = max(links, 1) * 2.0 * float(np.max(np.abs(o.populations())))
    err = max(np.max(np.abs(gfx - ofx)), np.max(np.abs(gfy - ofy))) / sc
    print(f"{spec[0]}: momentum exchange {ofx} {ofy}, rel {err:.2e}", flush=True)
    assert err <= TOL64


def test_largest_lattice_the_abi_accepts(gpu):
    """Edge of the 32-bit plane offsets: the largest 16384-wide lattice create accepts (9 planes of
    just under 2^31 / 9 elements, 8.6 GB per FP32 buffer) runs a uniform periodic flow that stays
    uniform with its mass kept; one more row is refused.  Zero steps is a no-op."""
    from paper_1812_05401_amd import binding as B
    nx = 16384
    ny = ((1 << 31) - 64 * 9) // (9 * nx)
    while nx * ny * 9 + 64 * 9 >= (1 << 31):
        ny -= 1
    with pytest.raises(B.VplbmError):
        B.vplbm_create(B.make_config(nx, ny + 1))
    case = I.Case("largest", nx, ny, storage="f32", bc=I.ALL_PERIODIC, u0=(0.02, -0.01), tau=0.8)
    s = gpu_sim(case)
    s.step(0)
    assert s.steps_done == 0
    s.step(2)
    obs = s.observables()
    s.close()
    assert obs["status"] == 0 and obs["step"] == 1
    assert abs(obs["mass"] / (nx * ny) - 1.0) < 1e-6
