"""Pins for the oracle's constants and single-node operators (CPU only).

Each check ties the oracle to something other than its own formulas: an identity the paper's
equations imply, a second printed equation, exact rational arithmetic, or a textbook property.
"""
from fractions import Fraction as Fr
import math

import numpy as np
import pytest

import oracle as O


def rng(seed=0):
    return np.random.default_rng(seed)


EPS = np.finfo(float).eps


def close(a, b, ulps=8):
    """Equal up to a few roundings of the largest entry (the scale of the populations)."""
    a, b = np.asarray(a), np.asarray(b)
    return np.max(np.abs(a - b)) <= ulps * EPS * max(np.max(np.abs(b)), 1e-300)


# ---- Eq. 3 / Eq. 5: velocity set and weights ---------------------------------------------

def test_velocity_set_is_d2q9():
    xi, _ = O.lattice()
    # nine distinct integer vectors covering {-1, 0, 1}^2, rest particle first
    assert {tuple(v) for v in xi} == {(a, b) for a in (-1, 0, 1) for b in (-1, 0, 1)}
    assert tuple(xi[0]) == (0, 0)
    # axis links 1..4 and diagonal links 5..8, each group ordered counter-clockwise from the
    # first quadrant (Eq. 3: angle (alpha-1) pi/2 and (2 alpha - 9) pi/4)
    ang = [math.atan2(v[1], v[0]) % (2 * math.pi) for v in xi]
    assert all(abs(xi[a]).sum() == 1 for a in range(1, 5))
    assert all(abs(xi[a]).sum() == 2 for a in range(5, 9))
    assert ang[1:5] == sorted(ang[1:5]) and ang[5:9] == sorted(ang[5:9])


def test_weights_satisfy_isotropy():
    xi, w = O.lattice()
    # exact rational identities that fix the D2Q9 weights (c_s^2 = 1/3)
    wf = [Fr(1, 9) * 4 if a == 0 else (Fr(1, 9) if a <= 4 else Fr(1, 36)) for a in range(9)]
    assert np.allclose(w, [float(x) for x in wf], rtol=0, atol=1e-17)
    assert sum(wf) == 1
    for i in range(2):
        assert sum(wf[a] * xi[a][i] for a in range(9)) == 0
        for j in range(2):
            assert sum(wf[a] * xi[a][i] * xi[a][j] for a in range(9)) == (Fr(1, 3) if i == j else 0)
            for k in range(2):
                assert sum(wf[a] * xi[a][i] * xi[a][j] * xi[a][k] for a in range(9)) == 0
                for l in range(2):
                    lhs = sum(wf[a] * xi[a][i] * xi[a][j] * xi[a][k] * xi[a][l] for a in range(9))
                    d = lambda p, q: 1 if p == q else 0
                    rhs = Fr(1, 9) * (d(i, j) * d(k, l) + d(i, k) * d(j, l) + d(i, l) * d(j, k))
                    assert lhs == rhs


def test_moment_matrix_rows_agree_with_velocity_set():
    """Rows 3 and 5 of Eq. 13 are the x and y velocity components of Eq. 3's numbering."""
    xi, _ = O.lattice()
    M = O.moment_matrix()
    assert np.array_equal(M[3], xi[:, 0]) and np.array_equal(M[5], xi[:, 1])
    assert np.array_equal(M[0], np.ones(9))


def test_moment_matrix_is_orthogonal():
    M = O.moment_matrix()
    G = M @ M.T
    assert np.array_equal(G, np.diag([9, 36, 36, 6, 12, 6, 12, 4, 4]).astype(float))


# ---- Eq. 4 and Eq. 12 ---------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(5))
def test_feq_moments(seed):
    r = rng(seed)
    rho, ux, uy = 1 + 0.1 * r.standard_normal(), 0.1 * r.standard_normal(), 0.1 * r.standard_normal()
    xi, _ = O.lattice()
    f = O.feq(rho, ux, uy)
    u = np.array([ux, uy])
    assert abs(f.sum() - rho) < 1e-15
    assert np.allclose(xi.T @ f, rho * u, rtol=0, atol=1e-16)
    P = np.einsum("a,ai,aj->ij", f, xi, xi)
    assert np.allclose(P, rho / 3 * np.eye(2) + rho * np.outer(u, u), rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", range(5))
def test_moment_equilibria_match_distribution_equilibria(seed):
    """Eq. 12 (printed moment equilibria) = M (Eq. 13) applied to f^eq (Eq. 4)."""
    r = rng(seed)
    rho, ux, uy = 1 + 0.1 * r.standard_normal(), 0.1 * r.standard_normal(), 0.1 * r.standard_normal()
    M = O.moment_matrix()
    assert np.allclose(M @ O.feq(rho, ux, uy), O.meq(rho, ux, uy), rtol=0, atol=2e-15)


# ---- Eq. 16 / Eq. 7: forcing moments -----------------------------------------------------

@pytest.mark.parametrize("seed", range(5))
def test_forcing_moments(seed):
    r = rng(seed)
    ux, uy, fx, fy = 0.1 * r.standard_normal(4)
    xi, _ = O.lattice()
    F = O.forcing(ux, uy, fx, fy)
    u, f = np.array([ux, uy]), np.array([fx, fy])
    tol = 16 * np.finfo(float).eps * np.abs(F).sum()   # rounding of a nine-term sum
    assert abs(F.sum()) < tol
    assert np.allclose(xi.T @ F, f, rtol=0, atol=tol)
    # second moment of the Guo/Lu term: u f + f u
    P = np.einsum("a,ai,aj->ij", F, xi, xi)
    assert np.allclose(P, np.outer(u, f) + np.outer(f, u), rtol=0, atol=tol)


# ---- Eqs. 17-18: penalized velocity and force --------------------------------------------

def _eq18_exact(f, chi, us, eta):
    """Eq. 18 and then Eq. 17, literally, in exact rational arithmetic (dt = 1)."""
    xi, _ = O.lattice()
    F = [Fr(x) for x in f]
    rho = sum(F)
    j = [sum(xi[a][i] * F[a] for a in range(9)) for i in range(2)]
    k = Fr(1, 2) * Fr(chi) / Fr(eta)
    u = [(j[i] + k * rho * Fr(us[i])) / (rho + k * rho) for i in range(2)]
    fpen = [-rho * Fr(chi) / Fr(eta) * (u[i] - Fr(us[i])) for i in range(2)]
    return rho, u, fpen


@pytest.mark.parametrize("eta", [1e-7, 1e-3, 1.0, 7.5])
@pytest.mark.parametrize("chi", [0, 1])
def test_vp_macro_matches_eq18_exactly(eta, chi):
    r = rng(int(eta * 1e7) % 97 + chi)
    for _ in range(4):
        f = O.feq(1 + 0.05 * r.standard_normal(), 0.05 * r.standard_normal(), 0.05 * r.standard_normal())
        f = f * (1 + 0.01 * r.standard_normal(9))
        us = 0.05 * r.standard_normal(2)
        rho, u, fp = O.vp_macro(f, chi, us, eta)
        rho_x, u_x, fp_x = _eq18_exact(f, chi, us, eta)
        assert abs(rho - float(rho_x)) <= 1e-15
        for i in range(2):
            assert abs(u[i] - float(u_x[i])) <= 1e-16
            # the force is well conditioned in the rewritten form: full relative accuracy
            assert abs(fp[i] - float(fp_x[i])) <= 1e-14 * max(abs(float(fp_x[i])), 1e-30) + 1e-300
        if chi == 0:
            assert fp[0] == 0 and fp[1] == 0


def test_vp_strong_penalization_limit():
    """As eta -> 0 the solid velocity is imposed and the force tends to -2 (j - rho u_s)."""
    f = O.feq(1.0, 0.04, -0.02)
    us = np.array([0.01, 0.03])
    rho, u, fp = O.vp_macro(f, 1, us, 1e-12)
    assert np.allclose(u, us, atol=1e-12)
    assert np.allclose(fp, -2 * (np.array([0.04, -0.02]) - rho * us), rtol=1e-10)


# ---- Eq. 2 + Eq. 7 (SRT) and Eq. 10 (MRT) --------------------------------------------------

def _random_node(seed):
    r = rng(seed)
    f = O.feq(1 + 0.05 * r.standard_normal(), 0.05 * r.standard_normal(), 0.05 * r.standard_normal())
    f = f * (1 + 0.02 * r.standard_normal(9))
    chi = int(seed % 2)
    us = 0.05 * r.standard_normal(2)
    eta = [1e-7, 0.3][seed % 3 == 0]
    rho, u, fp = O.vp_macro(f, chi, us, eta)
    return f, rho, u, fp


@pytest.mark.parametrize("seed", range(6))
def test_collisions_conserve_mass_and_add_the_force(seed):
    xi, _ = O.lattice()
    f, rho, u, fp = _random_node(seed)
    j = xi.T @ f
    outs = [O.collide_srt(f, rho, u, fp, 0.73)]
    for s in (O.mrt_rates(0.73, 3 / 16), O.mrt_rates(0.548, 3 / 8), rng(seed).uniform(0.1, 1.9, 9)):
        outs.append(O.collide_mrt(f, rho, u, fp, s))
    for g in outs:
        assert abs(g.sum() - rho) < 2e-15
        assert np.allclose(xi.T @ g, j + fp, rtol=0, atol=2e-15)


@pytest.mark.parametrize("seed", range(6))
def test_srt_relaxes_to_equilibrium_at_tau_one(seed):
    """tau = 1 without force: the post-collision state is f^eq of the node's moments."""
    f, rho, u, _ = _random_node(seed)
    g = O.collide_srt(f, rho, u, np.zeros(2), 1.0)
    assert close(g, O.feq(rho, u[0], u[1]))


@pytest.mark.parametrize("seed", range(6))
def test_mrt_inverse_matrix(seed):
    """All nine rates 1 and no force: g = M^-1 m^eq = f^eq, which needs M^-1 M = I."""
    f, rho, u, _ = _random_node(seed)
    g = O.collide_mrt(f, rho, u, np.zeros(2), np.ones(9))
    assert close(g, O.feq(rho, u[0], u[1]))
    # and zero rates without force leave f untouched
    assert close(O.collide_mrt(f, rho, u, np.zeros(2), np.zeros(9)), f, ulps=1)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("tau", [0.51, 0.8, 1.5, 10.0])
def test_mrt_with_equal_rates_is_srt(seed, tau):
    """The MRT model with every rate 1/tau is the SRT model, forcing included (Section 2.1.2)."""
    f, rho, u, fp = _random_node(seed)
    g_srt = O.collide_srt(f, rho, u, fp, tau)
    g_mrt = O.collide_mrt(f, rho, u, fp, np.full(9, 1 / tau))
    assert close(g_mrt, g_srt)
    # conserved-moment rates are irrelevant: Eq. 14's zeros with s_n = s_q = 1/tau also give SRT
    s = np.array([0, 1, 1, 0, 1, 0, 1, 1, 1]) / tau
    assert close(O.collide_mrt(f, rho, u, fp, s), g_srt)


def test_srt_optimum_is_lambda_three_eighths():
    """SRT has s_n = s_q = 1/tau, so Lambda = (tau - 1/2)^2; Lambda = 3/8 <=> tau = 1/2 + sqrt(6)/4."""
    tau = 0.5 + math.sqrt(6) / 4
    s = O.mrt_rates(tau, 3 / 8)
    assert np.allclose(s[[1, 2, 4, 6, 7, 8]], 1 / tau, rtol=1e-15)
    s = O.mrt_rates(0.7, 0.0016)
    lam = (1 / s[1] - 0.5) * (1 / s[4] - 0.5)
    assert abs(lam - 0.0016) < 1e-17


def _trt(f, rho, u, fp, sp, sm):
    """Two-relaxation-time form: symmetric parts relaxed with sp, antisymmetric with sm, forcing
    split the same way.  Written independently of the moment-space code."""
    xi, _ = O.lattice()
    opp = [int(np.where((xi == -xi[a]).all(1))[0][0]) for a in range(9)]
    fe = O.feq(rho, u[0], u[1])
    F = O.forcing(u[0], u[1], fp[0], fp[1])
    sym = lambda v: 0.5 * (v + v[opp])
    asym = lambda v: 0.5 * (v - v[opp])
    return (f - sp * sym(f - fe) - sm * asym(f - fe) + (1 - sp / 2) * sym(F) + (1 - sm / 2) * asym(F))


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("tau,lam", [(0.548, 3 / 16), (0.8, 3 / 8), (10.0, 0.0016), (0.7, 1.0)])
def test_mrt_equals_two_relaxation_time_form(seed, tau, lam):
    """Eq. 14 gives s_n to every even non-conserved moment and s_q to both odd ones, so Eq. 10 is
    a TRT collision; the moment-space oracle must agree with the TRT form to rounding."""
    f, rho, u, fp = _random_node(seed)
    s = O.mrt_rates(tau, lam)
    g = O.collide_mrt(f, rho, u, fp, s)
    assert close(g, _trt(f, rho, u, fp, s[1], s[4]))


# ---- velocity inlet -------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_zou_he_inlet_imposes_density_and_velocity(seed):
    r = rng(seed)
    xi, _ = O.lattice()
    f = O.feq(1.0, 0.05, 0.0) * (1 + 0.02 * r.standard_normal(9))
    U = (0.05 + 0.01 * r.standard_normal(), 0.01 * r.standard_normal())
    g = O.zou_he_inlet(f, *U)
    # the known populations are untouched
    assert np.array_equal(g[[0, 2, 3, 4, 6, 7]], f[[0, 2, 3, 4, 6, 7]])
    rho = g.sum()
    assert np.allclose(xi.T @ g, rho * np.array(U), rtol=0, atol=1e-16)
    # density from mass and normal momentum balance of the known populations
    known = f[0] + f[2] + f[4] + 2 * (f[3] + f[6] + f[7])
    assert abs(rho * (1 - U[0]) - known) < 1e-15
    # non-equilibrium bounce-back normal to the edge
    fe = O.feq(rho, *U)
    assert abs((g[1] - fe[1]) - (g[3] - fe[3])) < 1e-16


def test_body_motion_closed_form():
    b = O.make_body(O.DISK, cx=10, cy=20, r=3, ux=0.01, ay=2.0, freq=0.01)
    c, v = O.body_state(b, 25.0)   # quarter period: centre at the top of its stroke, at rest
    assert np.allclose(c, [10, 22], atol=1e-14) and np.allclose(v, [0.01, 0], atol=1e-15)
    c, v = O.body_state(b, 0.0)
    assert np.allclose(c, [10, 20]) and np.allclose(v, [0.01, 2 * math.pi * 0.01 * 2.0])
