"""Host post-processing (Eqs. 20, 22, 23) against closed forms."""
import math

import numpy as np

from paper_1812_05401_amd import analysis as A
from paper_1812_05401_amd import inputs as I


def test_strouhal_of_a_pure_sinusoid():
    u, d, st = 0.05, 64.0, 0.213
    period = d / (st * u)
    t = np.arange(60000)
    cl = 0.7 * np.sin(2 * math.pi * t / period + 0.3) + 0.05
    assert abs(A.strouhal(cl, d, u) / st - 1) < 1e-4
    assert A.strouhal(cl[:int(3 * period)], d, u) is None


def test_strouhal_ignores_rounding_noise():
    u, d, st = 0.05, 64.0, 0.2108
    period = d / (st * u)
    t = np.arange(50000)
    r = np.random.default_rng(1)
    cl = 0.46 * np.sqrt(2) * np.sin(2 * math.pi * t / period) + 0.05 * r.standard_normal(len(t))
    assert abs(A.strouhal(cl, d, u) / st - 1) < 2e-3


def test_force_coefficients_and_statistics():
    u, d = 0.05, 64.0
    q = 0.5 * u * u * d
    t = np.arange(20000)
    fx = q * (1.3 + 0.01 * np.sin(t / 300))
    fy = q * 0.9 * math.sqrt(2) * np.sin(2 * math.pi * t / 1000)
    s = A.wake_statistics(fx, fy, u, d)
    assert abs(s["C_Dave"] - 1.3) < 1e-3
    assert abs(s["C_Lrms"] - 0.9) < 1e-3
    assert abs(s["St"] - d / (1000 * u)) < 1e-6


def test_l2_error_matches_definition():
    r = np.random.default_rng(0)
    ua = r.normal(size=(5, 7))
    u = ua + 1e-3 * r.normal(size=(5, 7))
    w = r.random((5, 7)) < 0.6
    ref = math.sqrt(np.sum((u - ua)[w] ** 2) / np.sum(ua[w] ** 2))
    assert abs(A.l2_error(u, ua, w) - ref) < 1e-15
    v = np.stack([u, 2 * u])
    va = np.stack([ua, 2 * ua])
    assert abs(A.l2_error(v, va, w) - ref) < 1e-14


def test_spectral_strouhal_recovers_the_frequency_under_noise():
    """A 6400-step period over 50,000 samples: the periodogram peak gives St to 0.3%, with or
    without rounding-like noise of three times the signal's rms that defeats zero crossings."""
    n, period, d, u = 50_000, 6400.0, 64.0, 0.05
    t = np.arange(n)
    clean = 0.6 * np.sin(2 * np.pi * t / period + 0.3)
    st = d / (period * u)
    noisy = clean + np.random.default_rng(3).normal(0, 1.3, n)
    for cl in (clean, noisy):
        assert abs(A.strouhal_spectral(cl, d, u) / st - 1) < 3e-3
    assert A.strouhal_spectral(np.zeros(100), d, u) is None


def test_force_regions_add_up_to_the_next_steps_force():
    """The surface / interior split of the penalization force (study.body_force_regions), taken
    on a state, adds up to the force the oracle reduces in the next step."""
    import oracle as O
    from paper_1812_05401_amd import study
    from tests.helpers import oracle_sim
    case = I.cylinder_wake(160, 64, d=16.0, x0=40.0, re=100.0)
    o = oracle_sim(case)
    o.step(300)
    r = study.body_force_regions(o.populations(), o.mask(), 1, case.eta)
    o.step(1)
    ob = o.obs()
    sc = float(ob["fabs_sum"][0])
    assert r["surface_nodes"] > 0 and r["interior_nodes"] > 0
    assert abs(r["surface"][0] + r["interior"][0] - ob["fx"][0]) < 1e-12 * sc
    assert abs(r["surface"][1] + r["interior"][1] - ob["fy"][0]) < 1e-12 * sc
    assert abs(r["layers"][0][0] - r["surface"][0]) < 1e-14 * sc
    assert abs(sum(l[0] for l in r["layers"]) - ob["fx"][0]) < 1e-12 * sc
    assert sum(l[2] for l in r["layers"]) == r["surface_nodes"] + r["interior_nodes"]
