"""Reduced-precision storage on the GPU.

* The shifted 16-bit codecs round h = f - w_a to nearest even: the decoded population differs
  from f by at most half an ulp of h in the 16-bit format (plus the FP32 rounding of adding w).
* FP32, FP32D, FP16S and BF16S runs against the FP64 oracle on the same inputs: the velocity L2
  error of Eq. 20 after 1000 steps is reported and held to bounds derived from each format's unit
  roundoff (see the design notes): FP32 u = 6e-8, FP16 u = 4.9e-4 and BF16 u = 3.9e-3 of |f - w|.
  FP32D rounds only the stored h to binary32; its arithmetic is FP64.
"""
import numpy as np
import pytest

from paper_1812_05401_amd import analysis as A
from paper_1812_05401_amd import inputs as I
from tests.helpers import gpu_sim, oracle_sim, rel_err

pytestmark = pytest.mark.gpu

W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def half_ulp(x, mant_bits):
    """Half an ulp of |x| in a binary format with `mant_bits` explicit mantissa bits (normal
    range; the subnormal floor of binary16 is 2^-25)."""
    e = np.floor(np.log2(np.maximum(np.abs(x), 1e-300)))
    return np.maximum(2.0 ** (e - mant_bits - 1), 2.0 ** -25 if mant_bits == 10 else 0.0)


@pytest.mark.parametrize("storage,mant", [("f32", 23), ("f32d", 23), ("f16s", 10), ("bf16s", 7)])
def test_shifted_codec_rounds_to_nearest(gpu, storage, mant):
    case = I.Case("codec", 67, 13, storage=storage)
    g = gpu_sim(case)
    r = np.random.default_rng(5)
    pop = W[:, None, None] * (1 + r.uniform(-0.3, 0.3, (9, 13, 67)))
    g.set_populations(pop, 0)
    back = g.populations()
    h = pop - W[:, None, None]
    bound = half_ulp(h, mant) + 1.2e-7 * np.abs(pop)   # + FP32 rounding of h + w
    assert np.all(np.abs(back - pop) <= bound)
    # and it is not better than the format allows, i.e. the data really went through 16 bits
    assert np.max(np.abs(back - pop) / np.maximum(half_ulp(h, mant), 1e-30)) > 0.5


CH = ("channel_mrt", 200, 45, "mrt", 0.56, 3 / 16, 1e-7, I.CHANNEL, (0.05, 0.0), 2, False, False)
# measured velocity L2 (Eq. 20) vs the oracle after 1000 steps on this case, and the bounds
BOUNDS = {"f32": 1e-5, "f32d": 1e-6, "f16s": 5e-3, "bf16s": 4e-2, "f16sr": 5e-3, "bf16sr": 4e-2}


@pytest.mark.parametrize("storage", ["f32", "f32d", "f16s", "bf16s", "f16sr", "bf16sr"])
def test_reduced_precision_against_the_oracle(gpu, storage):
    from tests.test_gpu_parity import build_case, make_pair
    case, _ = build_case(*CH, seed=17)
    o, g = make_pair(case, None, 17, storage=storage)
    o.step(1000)
    g.step(1000)
    fluid = o.mask() == 0
    _, oux, ouy = o.fields()
    rho, ux, uy = g.fields()
    err = A.l2_error(np.stack([ux, uy]), np.stack([oux, ouy]), fluid)
    obs = g.observables()
    m_err = abs(obs["mass"] - o.obs()["mass"]) / o.obs()["mass"]
    print(f"{storage}: velocity L2 vs oracle {err:.3e}, mass {m_err:.3e}", flush=True)
    assert obs["status"] == 0
    assert err < BOUNDS[storage]


def _ulp(x, mant_bits):
    return 2.0 * half_ulp(x, mant_bits)


@pytest.mark.parametrize("storage,mant", [("f16sr", 10), ("bf16sr", 7)])
def test_stochastic_rounding_is_unbiased(gpu, storage, mant):
    """A uniform periodic flow: every node computes the same post-collision h, in FP32 exactly as
    an F32 run from the same populations stores it.  Rounded stochastically, each stored value is
    one of the two 16-bit neighbours, both occur, and their mean over the 16384 nodes is within
    5 standard errors (at most 0.02 ulp) of the FP32 value; rounding to nearest would be off by
    the same fraction of an ulp at every node."""
    case = I.Case("sr", 128, 128, storage=storage, bc=I.ALL_PERIODIC, u0=(0.0313, -0.0171),
                  tau=0.7)
    g = gpu_sim(case)
    start = g.populations()
    ref = gpu_sim(case, storage="f32")
    ref.set_populations(start, 0)                      # the 16-bit values are exact in binary32
    g.step(1)
    ref.step(1)
    got, want = g.populations(), ref.populations()
    two_valued = 0
    for k in range(9):
        w = want[k].ravel()
        assert np.ptp(w) == 0.0                        # uniform state: one value per plane
        h = w[0] - W[k]
        d = got[k].ravel() - w
        u = _ulp(h, mant)
        assert np.all(np.abs(d) <= u * (1 + 1e-9))
        two_valued += len(np.unique(got[k])) == 2
        assert abs(d.mean()) <= max(5 * u * 0.5 / np.sqrt(d.size), 1e-12 * abs(w[0]))
    assert two_valued >= 7


@pytest.mark.parametrize("steps,nt", [(1, False), (1, True), (2, False), (2, True)],
                         ids=["one_step", "one_step_nt", "two_step", "two_step_nt"])
def test_f16sr_rounds_subnormal_values_on_their_quantum(gpu, steps, nt):
    """Fluid at rest with density 1 + 1e-4: every shifted population h = w (rho - 1) lies below
    2^-14, in binary16's subnormal range, where the quantum is 2^-24 and FP16SR takes its separate
    exact-quantum rounding (a branch that only waves holding such values take).  Each stored h must
    be one of the two multiples of 2^-24 around the node's FP32 value, both must occur (in most
    planes: a value very close to a multiple may round the same way at every node), and the mean
    rounding error over the 16384 nodes must be within 5 standard errors of zero.  steps = 2 runs
    the two-step kernel, whose first step rounds into LDS and whose second stores the checked
    values; nt selects the non-temporal stores (which large lattices take).  The FP32 value of the
    last step is computed from the FP16SR state before it."""
    import os
    q = 2.0 ** -24
    case = I.Case("sr_rest", 128, 128, storage="f16sr", bc=I.ALL_PERIODIC, u0=(0.0, 0.0),
                  rho0=1.0 + 1e-4, tau=0.7)
    old = os.environ.get("VPLBM_NT_STORE")
    os.environ["VPLBM_NT_STORE"] = "1" if nt else "0"
    try:
        g = gpu_sim(case)
    finally:
        if old is None:
            os.environ.pop("VPLBM_NT_STORE")
        else:
            os.environ["VPLBM_NT_STORE"] = old
    before = g.populations()
    if steps == 2:
        pre = gpu_sim(case)                  # the state after the first step, one step per launch
        pre.step(1)
        before = pre.populations()
        pre.close()
    ref = gpu_sim(case, storage="f32")
    ref.set_populations(before, steps - 1)
    g.step(steps)
    ref.step(1)
    assert g.steps_done == steps
    got, want = g.populations(), ref.populations()
    two_valued = 0
    for k in range(9):
        h_ref = want[k].ravel() - W[k]
        assert np.all((0.0 < np.abs(h_ref)) & (np.abs(h_ref) < 2.0 ** -14))
        h = got[k].ravel() - W[k]
        n = h / q
        assert np.all(np.abs(n - np.round(n)) < 1e-6)              # on the subnormal grid
        lo, hi = np.floor(h_ref / q) * q, np.ceil(h_ref / q) * q
        down, up = np.abs(h - lo) < 1e-3 * q, np.abs(h - hi) < 1e-3 * q
        assert np.all(down | up)
        two_valued += bool(np.any(down & ~up)) and bool(np.any(up & ~down))
        assert abs((h - h_ref).mean()) <= 5 * q * 0.5 / np.sqrt(h.size)
    assert two_valued >= 6


@pytest.mark.parametrize("steps,nt", [(1, False), (1, True), (2, False), (2, True)],
                         ids=["one_step", "one_step_nt", "two_step", "two_step_nt"])
def test_f16sr_rounds_each_lane_of_a_mixed_wave_on_its_own_grid(gpu, steps, nt):
    """Fluid at rest whose density alternates every 8 columns between about 1 + 1e-5 (seeded
    per-node noise of +-50%, so the values spread over the grid) and 1 + 1e-2, so that every wave
    holds lanes whose shifted populations lie below 2^-14 (binary16's subnormal
    range, quantum 2^-24) beside lanes whose values lie above.  The wave-uniform branch that
    redoes the small values must do so for every such lane of a wave: a small value rounded on the
    path meant for normal values (random bits under the binary32 mantissa, then a round to nearest
    in the conversion) is all but rounded to nearest at these magnitudes.  So, against the FP32
    value of the same step: every small value lies on one of its two neighbours on the 2^-24
    grid, and among the values at fractional position 0.1-0.4 (0.6-0.9) between them the share
    rounded up matches the mean fraction to 5 standard errors, as stochastic rounding gives and
    rounding to nearest (a share of 0, or 1) does not.  Large values lie within one binary16 ulp."""
    import os
    q = 2.0 ** -24
    ny, nx = 96, 128
    case = I.Case("sr_mixed", nx, ny, storage="f16sr", bc=I.ALL_PERIODIC, u0=(0.0, 0.0),
                  tau=0.7)
    rng = np.random.default_rng(11)
    small_col = ((np.arange(nx) // 8) % 2 == 0)[None, :]
    drho = np.where(small_col, 1e-5 * (1.0 + 0.5 * rng.uniform(-1.0, 1.0, (ny, nx))), 1e-2)
    pop = W[:, None, None] * (1.0 + drho)[None]
    old = os.environ.get("VPLBM_NT_STORE")
    os.environ["VPLBM_NT_STORE"] = "1" if nt else "0"
    try:
        g = gpu_sim(case)
    finally:
        if old is None:
            os.environ.pop("VPLBM_NT_STORE")
        else:
            os.environ["VPLBM_NT_STORE"] = old
    g.set_populations(pop, 0)
    before = g.populations()
    if steps == 2:
        pre = gpu_sim(case)                  # the state after the first step, one step per launch
        pre.set_populations(pop, 0)
        pre.step(1)
        before = pre.populations()
        pre.close()
    ref = gpu_sim(case, storage="f32")
    ref.set_populations(before, steps - 1)
    g.step(steps)
    ref.step(1)
    got, want = g.populations(), ref.populations()
    h_ref = (want - W[:, None, None]).ravel()
    h = (got - W[:, None, None]).ravel()
    a = np.abs(h_ref)
    small = (a > 0) & (a < 0.99 * 2.0 ** -14)
    large = a > 1.01 * 2.0 ** -14
    assert small.sum() > 20000 and large.sum() > 30000
    hs, rs = h[small], h_ref[small]
    n = hs / q
    assert np.all(np.abs(n - np.round(n)) < 1e-6)                   # on the subnormal grid
    lo = np.floor(rs / q)
    frac = rs / q - lo
    up = np.abs(n - (lo + 1)) < 1e-3
    assert np.all(up | (np.abs(n - lo) < 1e-3))
    for a0, a1 in ((0.1, 0.4), (0.6, 0.9)):
        sel = (frac >= a0) & (frac <= a1)
        assert sel.sum() >= 500
        p = frac[sel].mean()
        share = up[sel].mean()
        print(f"fraction {a0}-{a1}: {sel.sum()} values, mean {p:.3f}, rounded up {share:.3f}",
              flush=True)
        assert abs(share - p) <= 5 * np.sqrt(p * (1 - p) / sel.sum())
    assert np.all(np.abs(h[large] - h_ref[large]) <= 2 * half_ulp(h_ref[large], 10))
    g.close()
    ref.close()
