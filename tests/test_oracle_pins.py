"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these checks re-types an oracle formula: each compares the oracle with
a closed form, a library routine, a brute-force integral of the continuum
definition (eq. C22_general), a number printed in the paper, or an invariant.
"""
import os

import numpy as np
import pytest
from scipy import integrate

import oracle
from paper_2607_00755_amd import inputs
from tests import mc_collision

HERE = os.path.dirname(os.path.abspath(__file__))


def kin(q, m=1.0):
    return q * q / (np.sqrt(q * q + m * m) + m)


def partner(pi, pn, pm, m=1.0):
    kt = kin(pn) + kin(pm) - kin(pi)
    return np.sqrt(kt * (kt + 2 * m))


# --------------------------------------------------------------------------
# Gauss-Legendre nodes (App. B): against numpy's routine.
def test_gauss_legendre_matches_numpy():
    for n in (1, 2, 5, 18, 64, 200):
        x, w = oracle.gauss_legendre(n)
        xr, wr = np.polynomial.legendre.leggauss(n)
        assert np.max(np.abs(x - xr)) < 1e-14
        assert np.max(np.abs(w - wr)) < 1e-13


# --------------------------------------------------------------------------
# P1: the paper's GL-in-mu / analytic-nu angular factor (eqs. app_I_mu,
# app_F_1d) converges to the closed form pi*S/(2 p_i) as N_mu grows.
@pytest.mark.parametrize("trip", [(1.0, 0.7, 1.4), (0.3, 0.5, 0.2), (2.0, 1.5, 3.0),
                                  (0.01, 0.02, 0.5), (5.0, 0.1, 5.2), (0.05, 3.0, 2.9)])
def test_angular_gl_converges_to_closed_form(trip):
    pi, pn, pm = trip
    ex = oracle.angular_exact(pi, partner(pi, pn, pm), pn, pm)
    errs = [abs(oracle.angular_gl(pi, pn, pm, nmu=k) - ex) / ex for k in (18, 100, 400)]
    assert errs[2] < 1e-2
    # converges (smooth cases reach machine precision already at N_mu = 100)
    assert errs[2] <= max(errs[0], 1e-12)


def test_discriminant_identity_exact():
    # The oracle evaluates b^2 - 4ac of eq. app_I_mu's quadratic
    # (a = -(K^2 + A1^2), b = -2 A0 A1, c = K^2 - A0^2) as
    # 4 K^2 (K^2 + A1^2 - A0^2); check the identity in exact rationals.
    from fractions import Fraction as Fr
    rng = np.random.default_rng(3)
    for _ in range(200):
        A0, A1, K2 = (Fr(int(v), 997) for v in rng.integers(-10**6, 10**6, 3))
        K2 = abs(K2)
        a, b, c = -(K2 + A1 * A1), -2 * A0 * A1, K2 - A0 * A0
        assert b * b - 4 * a * c == 4 * K2 * (K2 + A1 * A1 - A0 * A0)


def test_angular_closed_form_special_values():
    # All four momenta equal: S = 4p, Phi = 2 pi.
    for q in (0.1, 1.0, 7.0):
        assert abs(oracle.angular_exact(q, q, q, q) - 2 * np.pi) < 1e-12
    # Momenta that cannot close a triangle-pair give zero.
    assert abs(oracle.angular_exact(10.0, 0.1, 0.1, 0.1)) < 1e-14


# --------------------------------------------------------------------------
# P6: discrete gain (closed-form angular factor) against a brute-force Monte
# Carlo of the full continuum definition, Richardson-extrapolated in the grid.
def test_gain_matches_monte_carlo_of_definition():
    f = lambda q: inputs.bump_pair(q, 0.3, 1.5, 1.0, 0.5, 0.35, 0.35)
    picks = [3, 6, 9, 11]
    res = {}
    for n in (61, 121):
        p = inputs.log_grid(n, 1e-2, 20.0)
        op = oracle.Operator(p, quad=oracle.EXACT)
        _, g, _ = op.collision(f(p))
        k = (n - 1) // 15
        res[n] = g[[k * j for j in picks]]
    rich = res[121] + (res[121] - res[61]) / 3.0
    targets = inputs.log_grid(16, 1e-2, 20.0)[picks]
    for x, r in zip(targets, rich):
        mc, sd = mc_collision.gain(x, f, ns=2_000_000, seed=11)
        assert abs(r - mc) < 4.0 * sd + 2e-3 * mc, (x, r, mc, sd)


# --------------------------------------------------------------------------
# P2: the loss rate sum_j R_ij f_j against a deterministic 2-D quadrature of
# the continuum loss rate of eq. C22_general (MB input, T = 0.3); the error
# must fall like the square of the grid spacing.
def continuum_loss_rate(p1, f, m=1.0):
    e1 = np.sqrt(p1 * p1 + m * m)

    def inner(p2):
        e2 = np.sqrt(p2 * p2 + m * m)

        def ang(c):
            s = 2 * m * m + 2 * (e1 * e2 - p1 * p2 * c)
            ps = np.sqrt(max(s / 4 - m * m, 0.0))
            return ps / (4 * np.pi * np.sqrt(s))
        a, _ = integrate.quad(ang, -1.0, 1.0, epsabs=0, epsrel=1e-12)
        return 2 * np.pi * p2 * p2 / ((2 * np.pi) ** 3 * 2 * e2) * f(p2) * a

    val, _ = integrate.quad(inner, 0.0, 12.0, epsabs=0, epsrel=1e-11, limit=400)
    return val / (2 * e1)


def test_loss_rate_matches_continuum_integral():
    T = 0.3
    f = lambda q: np.exp(-np.sqrt(q * q + 1.0) / T)
    coarse = inputs.log_grid(49, 1e-3, 30.0)
    picks = [int(np.argmin(np.abs(coarse - x))) for x in (0.05, 0.3, 1.0, 3.0)]
    ref = np.array([continuum_loss_rate(coarse[i], f) for i in picks])
    rates = {}
    for n in (49, 97, 193):
        p = inputs.log_grid(n, 1e-3, 30.0)
        op = oracle.Operator(p, quad=oracle.EXACT)
        k = (n - 1) // 48
        rates[n] = (op.R @ f(p))[[k * i for i in picks]]
    e = {n: np.abs(rates[n] / ref - 1.0) for n in rates}
    # second order in the grid spacing ...
    assert np.all(e[97] < e[49] / 3.0) and np.all(e[193] < e[97] / 2.5), e
    # ... towards the continuum value (Richardson-extrapolated)
    rich = rates[193] + (rates[193] - rates[97]) / 3.0
    assert np.max(np.abs(rich / ref - 1.0)) < 2e-3, rich / ref - 1.0


# --------------------------------------------------------------------------
# P3: non-relativistic limit of the loss rate is n <sigma v> with
# sigma = |M|^2/(64 pi m^2); with |M|^2 = lambda^2 and m = 500 MeV this is the
# paper's tabulated sigma_T/m (golden fixture, App. A table).
def nr_sigma_from_oracle():
    T, m = 0.004, 1.0
    p = inputs.log_grid(97, 1e-4, 1.0)
    f = np.exp(-(np.sqrt(p * p + m * m) - m) / T)
    op = oracle.Operator(p, quad=oracle.EXACT, m2=1.0, mass=m)
    rate0 = (op.R @ f)[0]
    # n <v> for a particle at rest: int d^3p/(2pi)^3 f(p) p/E
    fv = lambda q: np.exp(-(np.sqrt(q * q + m * m) - m) / T) * q / np.sqrt(q * q + m * m)
    nv, _ = integrate.quad(lambda q: 4 * np.pi * q * q * fv(q) / (2 * np.pi) ** 3, 0, 1.0,
                           epsabs=0, epsrel=1e-12, limit=200)
    return rate0 / nv


def test_nr_cross_section_normalisation():
    sig = nr_sigma_from_oracle()
    assert abs(sig / (1.0 / (64 * np.pi)) - 1.0) < 1.5e-2


def test_sigma_over_m_matches_paper_table():
    sig_unit = nr_sigma_from_oracle() * (64 * np.pi)     # -> 1 up to the NR correction
    hbarc2_cm2_gev2 = 0.389379e-27
    gev_in_g = 1.78266192e-24
    m = 0.5
    rows = np.loadtxt(os.path.join(HERE, "golden", "sigma_T_over_m.txt"))
    for lam, tab in rows:
        sigma = sig_unit * lam * lam / (64 * np.pi * m * m)          # GeV^-2
        val = sigma * hbarc2_cm2_gev2 / (m * gev_in_g)               # cm^2/g
        assert abs(val / tab - 1.0) < 4e-2, (lam, val, tab)


# --------------------------------------------------------------------------
# P4: Maxwell-Boltzmann fixed point.  With the paper's log interpolation
# (eq. app_log_interp) C[z e^{-E/T}] vanishes term by term; with the linear
# interpolation of the precomputed form it vanishes at second order.
@pytest.mark.parametrize("z,T", [(1.0, 0.5), (3e-2, 2.0), (5.0, 0.2)])
def test_mb_fixed_point_log_interp(z, T):
    p = inputs.log_grid(24, 1e-2, 10.0)
    f = inputs.maxwell_boltzmann(p, 1.0, T, z)
    C, g, l = oracle.direct(p, f, quad=oracle.GL, nmu=18, interp=oracle.LOG)
    assert np.max(np.abs(C)) <= 1e-13 * np.max(np.abs(g))


def test_mb_fixed_point_lin_second_order():
    T = 0.5
    r = []
    for n in (32, 64, 128):
        p = inputs.log_grid(n, 1e-2, 10.0)
        op = oracle.Operator(p, quad=oracle.EXACT)
        C, g, _ = op.collision(inputs.maxwell_boltzmann(p, 1.0, T))
        r.append(np.max(np.abs(C)) / np.max(np.abs(g)))
    slopes = np.diff(np.log(r)) / np.log(2.0)
    assert np.all(slopes < -1.7) and np.all(slopes > -2.3), (r, slopes)


# --------------------------------------------------------------------------
# P5: the projection (App. C) removes the number and energy residuals; the raw
# residuals are reported and are non-zero.
def test_projection_conserves_number_and_energy():
    for n in (32, 96):
        p = inputs.log_grid(n, 1e-3, 1e2)
        op = oracle.Operator(p, quad=oracle.GL, nmu=18)
        f = inputs.two_bump_benchmark(p)
        C, _, _ = op.collision(f)
        Cp, d = op.project(f, C)
        h, E = op.grid.h, op.grid.E
        assert abs(np.sum(h * Cp)) <= 1e-14 * np.sum(h * np.abs(C)) * 10
        assert abs(np.sum(h * E * Cp)) <= 1e-14 * np.sum(h * E * np.abs(C)) * 10
        assert abs(d[2]) > 1e-6 and abs(d[3]) > 1e-6          # raw residuals non-zero
        assert abs(d[4]) < 1e-12 and abs(d[5]) < 1e-12
        # alpha, beta solve the 2x2 system of eq. app_projection_system
        xi = np.abs(f) / np.max(np.abs(f))
        xi[xi <= 1e-12] = 0
        M = np.array([[np.sum(h * xi), np.sum(h * E * xi)],
                      [np.sum(h * E * xi), np.sum(h * E * E * xi)]])
        rhs = np.array([np.sum(h * C), np.sum(h * E * C)])
        ab = np.linalg.solve(M, rhs)
        assert np.allclose(d[:2], ab, rtol=1e-8, atol=0)


def test_projection_leaves_conserving_operator_alone():
    p = inputs.log_grid(32, 1e-2, 10.0)
    op = oracle.Operator(p, quad=oracle.EXACT)
    f = inputs.bump_pair(p, 0.1, 2.0, 1.0, 0.5, 0.3, 0.3)
    C, _, _ = op.collision(f)
    Cp, _ = op.project(f, C)
    Cpp, d = op.project(f, Cp)
    assert np.max(np.abs(Cpp - Cp)) <= 1e-12 * np.max(np.abs(Cp))
    assert abs(d[0]) + abs(d[1]) < 1e-10 * (np.max(np.abs(C)) + 1e-300)


# --------------------------------------------------------------------------
# P7: direct per-(i,n,m) evaluation vs the precomputed A/R contraction.
@pytest.mark.parametrize("quad", [oracle.GL, oracle.EXACT])
def test_direct_equals_precomputed(quad):
    p = inputs.log_grid(40, 1e-3, 20.0)
    f = inputs.bump_pair(p, 0.2, 2.0, 1.0, 3.0, 0.3, 0.3)
    Cd, gd, ld = oracle.direct(p, f, quad=quad, nmu=18, interp=oracle.LIN)
    op = oracle.Operator(p, quad=quad, nmu=18)
    C, g, l = op.collision(f)
    sc = np.max(np.abs(g))
    assert np.max(np.abs(g - gd)) <= 1e-13 * sc
    assert np.max(np.abs(l - ld)) <= 1e-13 * sc
    assert np.max(np.abs(C - Cd)) <= 1e-13 * sc


# --------------------------------------------------------------------------
# P8: algebraic invariants.
def test_quadratic_scaling_and_single_bin():
    p = inputs.log_grid(32, 1e-2, 10.0)
    op = oracle.Operator(p, quad=oracle.GL)
    f = inputs.bump_pair(p, 0.1, 2.0, 1.0, 0.5, 0.3, 0.3)
    C1, _, _ = op.collision(f)
    C3, _, _ = op.collision(3.0 * f)
    assert np.max(np.abs(C3 - 9.0 * C1)) <= 1e-13 * np.max(np.abs(C3))
    k = 17
    e = np.zeros(32)
    e[k] = 2.0
    C, g, l = op.collision(e)
    assert np.allclose(g, op.A[:, k, k] * 4.0, rtol=1e-15, atol=0)
    assert np.all(l[np.arange(32) != k] == 0.0)
    assert abs(l[k] - 4.0 * op.R[k, k]) <= 1e-15 * abs(l[k])


def test_exact_kernel_symmetric_in_outgoing_pair():
    p = inputs.log_grid(48, 1e-3, 20.0)
    op = oracle.Operator(p, quad=oracle.EXACT)
    assert np.max(np.abs(op.A - op.A.transpose(0, 2, 1))) <= 1e-9 * np.max(op.A)


def test_cuts_and_brackets():
    p = inputs.log_grid(20, 1e-2, 5.0)
    op = oracle.Operator(p, quad=oracle.GL, keep_bracket=True)
    K = op.grid.K
    kt = (K[None, :, None] + K[None, None, :]) - K[:, None, None]
    keep = (kt >= K[0]) & (kt <= K[-1])
    assert np.array_equal(op.A > 0, keep & (op.A > 0))
    assert np.all(op.A[~keep] == 0.0)
    jl, wr = op.jl[keep], op.wr[keep]
    assert np.all((jl >= 0) & (jl <= 18))
    assert np.all((wr >= 0) & (wr <= 1))
    # the bracket reproduces the partner's kinetic energy
    assert np.allclose(K[jl] + wr * (K[jl + 1] - K[jl]), kt[keep], rtol=1e-13, atol=1e-300)
    # R rows sum to the total weight of their kept configurations
    assert np.allclose(op.R.sum(1), op.A.sum((1, 2)), rtol=1e-12)


# --------------------------------------------------------------------------
# P9: integrator orders (Sec. 4.2): RK4 error falls x16, Heun x4 per halving.
def test_rk4_and_heun_orders():
    w = inputs.single_fp64_n32()
    p = w.grid()
    op = oracle.Operator(p, quad=oracle.GL)
    f0 = w.f0()[0]
    g0 = op.gamma0(f0)
    T = 2.0 / g0
    ref = op.rk4(f0, 1.0, T / 256, 256)
    e = [np.max(np.abs(op.rk4(f0, 1.0, T / k, k) - ref)) for k in (8, 16)]
    assert 12.0 < e[0] / e[1] < 20.0, e
    hs = []
    for k in (16, 32):
        r = op.heun(f0, 1.0, 1.0, 0, 0, expansion=False, replay_dt=np.full(k, T / k))
        hs.append(np.max(np.abs(r["x"] - ref)))
    assert 3.0 < hs[0] / hs[1] < 5.0, hs


# --------------------------------------------------------------------------
# P10: H-theorem on the N=32 FP64 workload: entropy does not decrease along
# 100 RK4 steps of the projected operator; number and energy are conserved.
def test_entropy_non_decreasing_and_moments_conserved():
    w = inputs.single_fp64_n32()
    p = w.grid()
    op = oracle.Operator(p, quad=oracle.GL)
    f0 = w.f0()[0]
    dt = 0.1 / op.gamma0(f0)
    _, traj = op.rk4(f0, 1.0, dt, 100, traj=True)
    mom = np.array([op.moments(x) for x in np.vstack([f0, traj])])
    dN = np.abs(np.diff(mom[:, 0])) / np.abs(mom[:-1, 0])
    dE = np.abs(np.diff(mom[:, 1])) / np.abs(mom[:-1, 1])
    dS = np.diff(mom[:, 2])
    assert dN.max() <= 1e-12 and dE.max() <= 1e-12
    assert np.all(dS >= -1e-12 * np.abs(mom[:-1, 2]))
    assert mom[-1, 2] > mom[0, 2]


# --------------------------------------------------------------------------
# P11: Hubble drift.  An Euler step of one grid spacing in u shifts g by one
# bin exactly; the sum of V g changes only by the recorded outflow.
def test_drift_exact_shift_and_outflow():
    n = 40
    p = inputs.log_grid(n, 1e-3, 10.0)
    lnr = np.log(p[1] / p[0])
    dp_uniform = p * lnr
    g = inputs.bump_pair(p, 0.01, 1.0, 1.0, 0.5, 0.5, 0.5) * p ** 3
    d, out = oracle.drift(p, dp_uniform, g)
    shifted = g + lnr * d
    assert np.allclose(shifted[:-1], g[1:], rtol=1e-13, atol=1e-30)
    assert abs(shifted[-1]) <= 1e-13 * abs(g[-1])
    V = dp_uniform / p
    assert abs(np.sum(V * d) + out) <= 1e-13 * np.sum(np.abs(V * d))
    # default (trapezoid) widths: conservation net of outflow still exact
    gr = oracle.Grid(p)
    V2 = gr.dp / p
    d2, out2 = oracle.drift(p, gr.dp, g)
    assert abs(np.sum(V2 * d2) + out2) <= 1e-13 * np.sum(np.abs(V2 * d2))


def test_expansion_heun_conserves_comoving_number():
    n = 48
    p = inputs.log_grid(n, 1e-3, 20.0)
    op = oracle.Operator(p, quad=oracle.GL)
    f0 = inputs.bump_pair(p, 0.2, 2.0, 1.0, 1.0, 0.3, 0.3)
    x0 = f0 * p ** 3
    Hi = op.gamma0(f0)
    V = op.grid.dp / p
    tot0 = np.sum(V * x0)
    r = op.heun(x0, 3.0, Hi, 0.15, 1e-3, expansion=True, max_steps=4000)
    assert len(r["u"]) > 10 and abs(r["u"][-1] + r["dt"][-1] - 0.15) < 1e-12
    tot1 = np.sum(V * r["x"])
    assert abs(tot1 + r["outflow"] - tot0) <= 1e-12 * tot0 * len(r["u"])


# --------------------------------------------------------------------------
# Adaptive Heun controller (Sec. 4.2: Euler predictor, trapezoid corrector,
# their difference as the error estimate).  Started from a first step of
# half the interval, the controller must reject until the estimate falls
# to one; the end state, against a fine fixed-step RK4 solution of the same
# equation (dx/du = lambda C / H_i without expansion), must be within rtol
# and must improve in proportion to rtol; a second-order method needs
# about sqrt(100) = 10 times the steps for a 100 times tighter rtol.
def test_heun_controller_rejects_and_meets_tolerance():
    w = inputs.single_fp64_n32()
    p = w.grid()
    op = oracle.Operator(p, quad=oracle.GL)
    f0 = w.f0()[0]
    Hi = op.gamma0(f0)
    u_end = 2.0
    ref = op.rk4(f0, 1.0 / Hi, u_end / 4000, 4000)
    ref2 = op.rk4(f0, 1.0 / Hi, u_end / 2000, 2000)
    assert np.max(np.abs(ref - ref2)) <= 1e-12 * np.max(np.abs(ref))
    errs, steps = {}, {}
    for rtol in (1e-4, 1e-6):
        r = op.heun(f0, 1.0, Hi, u_end, 1.0, expansion=False, rtol=rtol, max_steps=100000)
        a = r["attempts"]
        assert r["rejected"] >= 3 and not a["accepted"][0]
        assert np.all(a["err"][a["accepted"]] <= 1.0)
        assert np.all(a["err"][~a["accepted"]] > 1.0)
        assert a["accepted"].sum() == len(r["dt"]) and (~a["accepted"]).sum() == r["rejected"]
        assert np.allclose(a["dt"][a["accepted"]], r["dt"], rtol=0, atol=0)
        assert abs(r["u"][-1] + r["dt"][-1] - u_end) <= 1e-13
        errs[rtol] = np.max(np.abs(r["x"] - ref)) / np.max(np.abs(ref))
        steps[rtol] = len(r["dt"])
        assert errs[rtol] <= rtol, (rtol, errs[rtol])
    assert errs[1e-6] <= errs[1e-4] / 30.0, errs
    assert 5.0 <= steps[1e-6] / steps[1e-4] <= 20.0, steps


def test_heun_step_size_law():
    """The step-size law both implementations take (the paper does not state
    one): dt_next = dt * clamp(0.9 err^-1/2, 0.2, 5), cut short only where
    the step would pass u_end.  A consistency check of that reading against
    the oracle's attempt log, not an independent pin: its accuracy is
    pinned by the test above."""
    w = inputs.single_fp64_n32()
    p = w.grid()
    op = oracle.Operator(p, quad=oracle.GL)
    f0 = w.f0()[0]
    Hi = op.gamma0(f0)
    r = op.heun(f0, 1.0, Hi, 2.0, 1.0, expansion=False, rtol=1e-5, max_steps=100000)
    a = r["attempts"]
    want = a["dt"][:-1] * np.clip(0.9 / np.sqrt(a["err"][:-1]), 0.2, 5.0)
    got = a["dt"][1:]
    free = got < want * (1 - 1e-12)            # shortened to end at u_end
    assert free.sum() <= 1
    assert np.allclose(got[~free], want[~free], rtol=1e-14, atol=0)


# --------------------------------------------------------------------------
# Hubble rate in the collision term of eq. numerical_evolution_loga: with
# g = a^3 p^3 f, the collision part of dg/du is a^3 p^3 lambda C[f] / H.
# For the same g, f scales as a^-3, so C[f] as a^-6, while a^3/H = a^5/H_i
# in the radiation era (H = H_i a^-2): the collision increment of one tiny
# step started at u = 1 is e^-1 times the one started at u = 0.  At u = 0
# (a = 1) it is dt p^3 lambda C[f] / H_i to first order in dt.
def test_expansion_collision_term_scales_with_hubble_rate():
    w = inputs.single_fp64_n32()
    p = w.grid()
    op = oracle.Operator(p, quad=oracle.GL)
    f0 = w.f0()[0]
    Hi = op.gamma0(f0)
    g0 = f0 * p ** 3
    dt = 1e-7

    def collision_increment(u0, lam):
        step = lambda l: op.heun(g0, l, Hi, 0.0, 0.0, expansion=True, replay_dt=[dt], u0=u0)["x"]
        return step(lam) - step(0.0)

    d0 = collision_increment(0.0, 2.0)
    d1 = collision_increment(1.0, 2.0)
    scale = np.max(np.abs(d0))
    assert np.max(np.abs(d1 - np.exp(-1.0) * d0)) <= 1e-6 * scale
    C = op.collision(f0, project=True)[0]
    assert np.max(np.abs(d0 - dt * 2.0 * p ** 3 * C / Hi)) <= 1e-5 * scale


# --------------------------------------------------------------------------
# P14: on the paper's two-bump input with N_mu = 18 the projection changes C
# by less than one per cent of max|C_raw| (App. C, pointwise figure).
@pytest.mark.parametrize("n", [96, 256])
def test_projection_pointwise_correction_below_percent(n):
    p = inputs.log_grid(n, 1e-3, 1e2)
    op = oracle.Operator(p, quad=oracle.GL, nmu=18)
    f = inputs.two_bump_benchmark(p)
    C, _, _ = op.collision(f)
    Cp, d = op.project(f, C)
    assert np.max(np.abs(Cp - C)) < 1e-2 * np.max(np.abs(C))
    assert d[6] < 5e-2 and d[7] < 5e-2


# --------------------------------------------------------------------------
# Quantum statistics (eq. Lambda_quantum): the direct evaluation with
# Bose-Einstein / Fermi-Dirac factors against the Monte Carlo of the same
# continuum integral, Richardson-extrapolated in the grid; eta = 0 is the
# dilute operator.
@pytest.mark.parametrize("eta,amp", [(1, 1.0), (-1, 0.9)])
def test_quantum_operator_matches_monte_carlo(eta, amp):
    f = lambda q: inputs.bump_pair(q, 0.3, 1.5, amp, 0.5 * amp, 0.35, 0.35)
    picks = [4, 8, 11]
    res = {}
    for n in (61, 121):
        p = inputs.log_grid(n, 1e-2, 20.0)
        _, g, l = oracle.direct(p, f(p), quad=oracle.EXACT, interp=oracle.LIN, eta=eta)
        k = (n - 1) // 15
        idx = [k * j for j in picks]
        res[n] = (g[idx], l[idx])
    targets = inputs.log_grid(16, 1e-2, 20.0)[picks]
    for t, x in enumerate(targets):
        (mg, sg), (ml, sl) = mc_collision.collision(x, f, eta, ns=2_000_000, seed=17 + t)
        rg = res[121][0][t] + (res[121][0][t] - res[61][0][t]) / 3.0
        rl = res[121][1][t] + (res[121][1][t] - res[61][1][t]) / 3.0
        assert abs(rg - mg) < 4.0 * sg + 3e-3 * mg, (x, rg, mg, sg)
        assert abs(rl - ml) < 4.0 * sl + 3e-3 * ml, (x, rl, ml, sl)


def test_quantum_operator_dilute_limit_and_statistics_sign():
    p = inputs.log_grid(28, 1e-2, 10.0)
    f = inputs.bump_pair(p, 0.2, 2.0, 0.8, 0.4, 0.3, 0.3)
    c0, g0, l0 = oracle.direct(p, f, interp=oracle.LOG)
    cd, gd, ld = oracle.direct(p, f, interp=oracle.LOG, eta=0)
    assert np.array_equal(c0, cd)
    cb, gb, lb = oracle.direct(p, f, interp=oracle.LOG, eta=1)
    cf, gf, lf = oracle.direct(p, f, interp=oracle.LOG, eta=-1)
    # Bose enhancement raises both rates, Pauli blocking lowers them
    assert np.all(gb >= g0) and np.all(gf <= g0) and np.all(lb >= l0) and np.all(lf <= l0)
    # the eta-odd parts are equal and opposite (the eta^2 terms cancel in Lambda)
    assert np.allclose((cb - c0), -(cf - c0), rtol=1e-10, atol=1e-14 * np.max(np.abs(gb)))


# --------------------------------------------------------------------------
# Freeze-in sources of the two-source scenario (Sec. 3) and the two regimes
# of the evolution (Sec. 4.2).
def test_condensate_deposit_injects_number_and_energy():
    """The condensate injects 2 Gamma nu particles per unit time at energy
    E0 = sqrt(p0^2 + m^2) each (number and energy injection rates
    C_0 = 2 Gamma n, C_E = 2 E0 Gamma n of Sec. 3): the deposit on the grid
    must carry exactly both moments, at any p0 inside the grid."""
    p = inputs.log_grid(40, 1e-3, 20.0)
    op = oracle.Operator(p)
    h, E = op.grid.h, op.grid.E
    Hi, N0, Gam, u = 1.0, 0.7, 0.4, 0.3
    nu = np.exp(-3 * u) * N0 * np.exp(-(Gam / (2 * Hi)) * (np.exp(2 * u) - 1))
    for p0 in (2e-3, 0.05, 0.8, float(p[17]), 7.3, 19.9):
        S = op.sources(u, Hi, N0=N0, Gamma=Gam, p0=p0)
        assert np.count_nonzero(S) <= 2 and np.all(S >= 0)
        E0 = np.sqrt(p0 * p0 + 1.0)
        assert abs(np.sum(h * S) / (2 * Gam * nu) - 1) < 1e-13
        assert abs(np.sum(h * E * S) / (2 * Gam * nu * E0) - 1) < 1e-13
        j = int(np.flatnonzero(S)[0])
        assert p[j] <= p0 * (1 + 1e-12) and (np.count_nonzero(S) == 1 or p0 <= p[j + 1])
    assert op.deposit(30.0)[0] == -1 and op.deposit(1e-4)[0] == -1


def test_condensate_decay_law():
    """a^3 n_Phi from the closed form against a numerical solution of the
    decay law dn/dt + 3 H n = -Gamma n written in u = ln a,
    d(a^3 n)/du = -(Gamma / H(u)) a^3 n, H = H_i e^{-2u}."""
    from scipy.integrate import solve_ivp
    Hi, N0 = 2.0, 1.3
    for Gam in (0.05, 1.0, 6.0):
        sol = solve_ivp(lambda u, y: -(Gam / (Hi * np.exp(-2 * u))) * y, (0.0, 1.5), [N0],
                        rtol=1e-12, atol=1e-300, dense_output=True, method="DOP853")
        for u in (0.1, 0.5, 1.0, 1.5):
            ref = float(sol.sol(u)[0])
            got = oracle.condensate_a3nu(N0, Gam, Hi, u)
            assert abs(got - ref) <= 1e-9 * N0, (Gam, u, got, ref)


def test_higgs_source_rate_closed_form():
    """The number injection of eq. C_higgs_decay, int p^2 C_h dp, has the
    closed form kappa T sqrt(m_h^2 - 4 m^2) K1(m_h / T) (the thermal average
    of a decay in a Maxwell-Boltzmann bath); the discrete sum_i h_i S_i
    matches it to rounding on a grid that covers the source's support (the
    trapezoid rule in ln p of a smooth integrand that vanishes at both ends
    converges faster than any power of the spacing)."""
    from scipy.special import k1
    kappa, mh = 0.37, 5.0
    for T in (0.8, 2.0):
        ref = kappa * T * np.sqrt(mh * mh - 4.0) * k1(mh / T)
        for n in (100, 400):
            g = oracle.Grid(inputs.log_grid(n, 1e-6, 200.0))
            # Ti such that T(u) = Ti e^{-u} equals T at u = 0.3
            S = oracle.sources(g, 0.3, 1.0, kappa=kappa, mh=mh, Ti=T * np.exp(0.3))
            assert np.all(S >= 0)
            assert abs(np.sum(g.h * S) / ref - 1.0) < 1e-12, (T, n)


def test_gamma22_is_n_sigma_vrel_nonrelativistic():
    """Gamma_22 = n <sigma v> (Sec. 4.2): for a non-relativistic
    Maxwell-Boltzmann f the mean relative speed is sqrt(16 T / (pi m)) and
    sigma = |M|^2 / (64 pi m^2), n = int d^3p/(2 pi)^3 f; the rate prefactor
    lambda multiplies it; f -> c f scales it by c."""
    T, m = 0.004, 1.0
    p = inputs.log_grid(97, 1e-4, 1.0)
    f = np.exp(-(np.sqrt(p * p + m * m) - m) / T)
    op = oracle.Operator(p, quad=oracle.EXACT, m2=1.0, mass=m)
    n_ref, _ = integrate.quad(lambda q: 4 * np.pi * q * q * np.exp(-(np.sqrt(q * q + 1) - 1) / T)
                              / (2 * np.pi) ** 3, 0, 1.0, epsabs=0, epsrel=1e-12, limit=200)
    ref = n_ref * np.sqrt(16 * T / (np.pi * m)) / (64 * np.pi)
    assert abs(op.gamma22(f) / ref - 1.0) < 1.5e-2
    assert abs(op.gamma22(f, lam=3.0) / op.gamma22(f) - 3.0) < 1e-13
    assert abs(op.gamma22(2.5 * f) / op.gamma22(f) - 2.5) < 1e-13
    assert op.gamma22(np.zeros_like(f)) == 0.0


def _freeze_in_setup(n=40):
    p = inputs.log_grid(n, 1e-3, 20.0)
    return p, oracle.Operator(p)


def test_freeze_in_source_only_conserves_total_number():
    """Source-only regime: the comoving number of chi, the number drifted out
    below p_min and twice the condensate's a^3 n_Phi add up to a constant
    (each decay gives two chi); fixed-step RK4 keeps it to fourth order."""
    p, op = _freeze_in_setup()
    V = op.grid.dp / p
    Hi, N0, Gam, p0 = 1.0, 1.0, 0.6, 0.8
    x0 = inputs.bump_pair(p, 0.5, 2.0, 1e-3, 5e-4, 0.3, 0.3) * p ** 3
    inv0 = np.sum(V * x0) + 2 * N0
    errs = []
    for du in (0.04, 0.02, 0.01):
        r = op.freeze_in(x0, 0.0, Hi, 1.2, du, N0=N0, Gamma=Gam, p0=p0)
        assert r["n_src"] == int(round(1.2 / du)) and len(r["u"]) == 0
        inv = np.sum(V * r["x"]) + r["outflow"] + 2 * oracle.condensate_a3nu(N0, Gam, Hi, 1.2)
        errs.append(abs(inv - inv0) / inv0)
    assert errs[-1] < 1e-9, errs
    assert 10.0 < errs[0] / errs[1] < 24.0 and 10.0 < errs[1] / errs[2] < 24.0, errs


def test_freeze_in_switch_fires_at_threshold():
    """The elastic operator is switched on at the first step whose state has
    Gamma_22 / H > eps_switch, and not before."""
    p, op = _freeze_in_setup()
    Hi, N0, Gam, p0, du, eps = 1.0, 2.0, 0.5, 0.8, 0.02, 1e-2
    x0 = np.zeros(len(p))
    lam = 150.0
    r = op.freeze_in(x0, lam, Hi, 1.5, du, eps_switch=eps, N0=N0, Gamma=Gam, p0=p0,
                     max_steps=20000)
    k = r["n_src"]
    assert 5 < k < 70 and abs(r["u_switch"] - k * du) < 1e-12 and len(r["u"]) > 0

    def state(steps):
        s = op.freeze_in(x0, lam, Hi, 1.5, du, eps_switch=eps, N0=N0, Gamma=Gam, p0=p0,
                         max_steps=steps)
        assert s["n_src"] == steps and len(s["u"]) == 0
        u = steps * du
        return op.gamma22(s["x"] / (np.exp(3 * u) * p ** 3), lam) / (Hi * np.exp(-2 * u))

    assert state(k) > eps >= state(k - 1)


def test_freeze_in_regime_two_is_the_heun_of_the_expanding_run():
    """With the switch at the start and no sources, the second regime is the
    adaptive Heun of the expanding-universe equation, step for step."""
    p, op = _freeze_in_setup()
    f0 = inputs.bump_pair(p, 0.2, 2.0, 1.0, 1.0, 0.3, 0.3)
    x0 = f0 * p ** 3
    Hi = op.gamma0(f0)
    a = op.heun(x0, 3.0, Hi, 0.1, 1e-3, expansion=True, max_steps=4000)
    b = op.freeze_in(x0, 3.0, Hi, 0.1, 0.01, eps_switch=-1.0, dt0=1e-3, max_steps=4000)
    assert b["n_src"] == 0 and b["u_switch"] == 0.0
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["dt"], b["dt"])


def test_freeze_in_with_collisions_conserves_total_number():
    """Both regimes with the condensate source: comoving chi number +
    outflow + 2 a^3 n_Phi stays constant to the integrators' tolerance
    (the projected elastic operator conserves number)."""
    p, op = _freeze_in_setup()
    V = op.grid.dp / p
    Hi, N0, Gam, p0 = 1.0, 2.0, 0.5, 0.8
    x0 = np.zeros(len(p))
    r = op.freeze_in(x0, 150.0, Hi, 1.0, 0.02, N0=N0, Gamma=Gam, p0=p0, max_steps=20000)
    assert r["n_src"] > 0 and len(r["u"]) > 0 and abs(r["u"][-1] + r["dt"][-1] - 1.0) < 1e-12
    inv = np.sum(V * r["x"]) + r["outflow"] + 2 * oracle.condensate_a3nu(N0, Gam, Hi, 1.0)
    assert abs(inv - 2 * N0) < 1e-7 * 2 * N0, inv - 2 * N0


# --------------------------------------------------------------------------
# The comoving grid of Sec. 4.1 (q = a p fixed, the operator of the grid
# q / a at each a): scaling limits, the tabulated reading, conservation.
def test_comoving_operator_scaling_limits():
    """For fixed f on the q grid the operator scales as a^-1 when the
    particles are massless (every weight is homogeneous of degree -1 in the
    momenta and the cut pattern is scale free) and as a^-4 when they are
    non-relativistic (E = m, K = p^2 / 2m)."""
    for mass, lo, hi, power in ((1e-7, 1e-2, 10.0, 1), (1.0, 1e-6, 1e-4, 4)):
        q = inputs.log_grid(24, lo, hi)
        f = inputs.bump_pair(q, np.sqrt(lo * hi) / 3, np.sqrt(lo * hi) * 3, 1.0, 0.5, 0.3, 0.3)
        c = oracle.Comoving(q, mass=mass)
        C0 = c.collision(f, 0.0, project=False)
        for u in (0.3, 1.0):
            Cu = c.collision(f, u, project=False)
            assert np.max(np.abs(Cu * np.exp(power * u) - C0)) <= 1e-8 * np.max(np.abs(C0)), (mass, u)


def test_comoving_tabulation_is_exact_at_nodes_and_first_order_between():
    """Tabulating the tensors over u = ln a reproduces the exact operator at
    the nodes, but between nodes converges only at first order: the grid
    range cuts switch entries of A on and off as a changes, so A(a) jumps.
    (This is why the evolution keeps the fixed physical grid with drift.)"""
    q = inputs.log_grid(24, 1e-2, 10.0)
    f = inputs.bump_pair(q, 0.2, 2.0, 1.0, 0.5, 0.3, 0.3)
    ex = oracle.Comoving(q)
    us = np.linspace(0.013, 0.987, 11)
    refs = [ex.collision(f, u) for u in us]
    errs = []
    for J in (5, 17, 33):
        t = oracle.Comoving(q, ntab=J, umin=0.0, umax=1.0)
        for j in (0, J // 2, J - 1):
            assert np.array_equal(t.collision(f, j * t.du), ex.collision(f, j * t.du))
        errs.append(max(np.max(np.abs(t.collision(f, u) - r)) / np.max(np.abs(r))
                        for u, r in zip(us, refs)))
    assert errs[0] > errs[1] > errs[2] > 5e-3, errs


def test_comoving_heun_conserves_comoving_number():
    """a^3 sum_i h_i(a) f_i = sum_i q_i^2 dq_i f_i is constant along the
    comoving evolution: every stage of the projected operator conserves the
    number moment of its own grid, and h(a) = q^2 dq / a^3."""
    q = inputs.log_grid(24, 1e-2, 10.0)
    f0 = inputs.bump_pair(q, 0.2, 2.0, 1.0, 0.5, 0.3, 0.3)
    c = oracle.Comoving(q)
    g = c.grid(0.0)
    w = g.h                     # q^2 dq at a = 1
    Hi = oracle.Operator(q).gamma0(f0)       # time in units of the initial loss rate
    r = c.heun(f0, 2.0, Hi, 0.2, 1e-3, max_steps=5000)
    assert len(r["u"]) > 5 and abs(r["u"][-1] + r["dt"][-1] - 0.2) < 1e-12
    assert abs(np.sum(w * r["x"]) / np.sum(w * f0) - 1.0) < 1e-12
    assert np.max(np.abs(r["x"] - f0)) > 1e-3 * np.max(f0)       # it did evolve
