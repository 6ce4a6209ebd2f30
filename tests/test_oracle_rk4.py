"""Pins of the oracle's RK4 substeps (classic four-stage Runge-Kutta, each
substep over dt with its boundary data frozen).  Each test checks the RK4
path against something other than itself: the full-tensor S_N scheme with
the same integrator, the fourth-degree Taylor factor of a scalar decay, the
exponential flow, and the observed order of accuracy.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import workloads as wk
from oracle import ddlra as dd
from oracle import sn_full as sn

from test_oracle_pins import full_rank_case, neighbour_inflow, rel, sub_block, SubGrid


def taylor4(z):
    return 1.0 + z + z * z / 2.0 + z ** 3 / 6.0 + z ** 4 / 24.0


@pytest.mark.parametrize("axis", [0, 1])
def test_rk4_full_rank_kstep_equals_sn_with_frozen_inflow(axis):
    """At full angular rank the RK4 K-step of every subdomain is the S_N
    upwind scheme advanced by one RK4 step on that subdomain alone, with the
    neighbours' cells frozen at their start-of-stage values."""
    wl = full_rank_case()
    wl.integrator = "rk4"
    prob = dd.Problem(wl)
    state = dd.initial_state(wl)
    F0 = sn.from_flat(dd.assemble(state, prob), wl)
    recs = []
    dd.stage_advect(state, axis, prob, records=recs)
    for s, rec in enumerate(recs):
        g = SubGrid(wl, prob, s)
        lo, hi = neighbour_inflow(F0, prob, s, axis)
        Fs = sub_block(F0, prob, s).reshape(prob.lny, prob.lnx, -1)
        ref = sn._rk4(lambda X: sn.advect_operator(X, axis, g, lo, hi), Fs, prob.dt)
        got = rec["K1"] @ rec["V_hat"].T
        assert rel(got, ref.reshape(prob.N, -1)) < 1e-12
        # and it is not the Euler step
        eul = Fs + prob.dt * sn.advect_operator(Fs, axis, g, lo, hi)
        assert rel(got, eul.reshape(prob.N, -1)) > 1e-6


def test_rk4_pure_absorption_factor():
    """c_s = 0, Q = 0, uniform sigma_a: the collision stage multiplies F by
    T4(-x) T4(x) T4(-x), x = dt sigma_a, T4 the degree-4 Taylor polynomial of
    exp (K-step forward, S-step backward, L-step forward), at any rank."""
    n = 8 * 8
    sa = 2.7
    wl = wk.make_custom(8, 8, 2, 2, wk.product_directions(4, 4), [3, 4, 2, 5], seed=2,
                        sigma_a=np.full(n, sa), cfl=0.5)
    wl.integrator = "rk4"
    prob = dd.Problem(wl)
    state = dd.initial_state(wl)
    out = dd.stage_collision(state, prob)
    x = prob.dt * sa
    fac = taylor4(-x) * taylor4(x) * taylor4(-x)
    for (U, S, V), (U1, S1, V1) in zip(state, out):
        assert rel(U1 @ S1 @ V1.T, fac * (U @ S @ V.T)) < 1e-14


def test_rk4_pure_absorption_converges_fourth_order():
    """Whole steps with c_adv = 0: F(T) -> exp(-sigma_a T) F(0) with error
    ratio 16 on halving dt."""
    errs = []
    sa, T = 1.5, 0.4
    for nst in (8, 16, 32):
        wl = wk.make_custom(4, 4, 2, 2, wk.product_directions(4, 4), [2] * 4, seed=4,
                            sigma_a=np.full(16, sa), c_adv=0.0, r_int_max=6, r_fixed=2)
        wl.integrator = "rk4"
        wl.dt = T / nst
        prob = dd.Problem(wl)
        state = dd.initial_state(wl)
        F0 = dd.assemble(state, prob)
        for _ in range(nst):
            state = dd.dd_step(state, prob)
        errs.append(rel(dd.assemble(state, prob), math.exp(-sa * T) * F0))
    assert 14.0 < errs[0] / errs[1] < 18.0 and 14.0 < errs[1] / errs[2] < 18.0, errs


def _exact_affine_flow(f, y0, dt):
    """exp flow of the affine ODE y' = f(y) over dt, from its matrix form
    (f(0) and the images of the unit matrices) and scipy's expm."""
    shp = y0.shape
    n = y0.size
    b = f(np.zeros(shp)).ravel()
    A = np.empty((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        A[:, k] = f(e.reshape(shp)).ravel() - b
    Z = np.zeros((n + 1, n + 1))
    Z[:n, :n] = A
    Z[:n, n] = b
    y = scipy.linalg.expm(dt * Z) @ np.append(y0.ravel(), 1.0)
    return y[:n].reshape(shp)


@pytest.mark.parametrize("axis", [0, 1])
def test_rk4_kstep_local_error_is_fifth_order(axis):
    """One low-rank K-step: the RK4 result against the exact flow of the same
    frozen-boundary ODE; halving dt divides the error by about 32."""
    errs = []
    for cfl in (0.2, 0.1):
        wl = wk.make_custom(8, 8, 2, 2, wk.product_directions(4, 4), [3] * 4, seed=9, cfl=cfl)
        wl.integrator = "rk4"
        prob = dd.Problem(wl)
        recs = []
        dd.stage_advect(dd.initial_state(wl), axis, prob, records=recs)
        e = []
        for rec in recs:
            f = lambda K: dd.kstep_rhs(K, rec["P"], rec["lam"], rec["Kb_lo"], rec["Kb_hi"], axis, prob)
            ex = _exact_affine_flow(f, rec["K0"], prob.dt)
            e.append(rel(rec["K1"], ex))
        errs.append(max(e))
    assert 24.0 < errs[0] / errs[1] < 40.0, errs


def test_rk4_advection_s_and_l_steps_local_error_is_fifth_order():
    """The advection S- and L-step RK4 results against the exact flows of
    the Euler right-hand sides of the same stage (S' = -h^2 U1^T A(U1 S),
    L' = (h^2 U1^T A_dir(U1 L^T))^T with the frozen ghosts): halving dt
    divides the local error by about 32, so the RK4 stages integrate the
    same right-hand sides as the Euler substeps (a sign or transpose slip in
    either would leave an O(dt) or O(1) gap instead)."""
    errs = []
    for cfl in (0.2, 0.1):
        wl = wk.make_custom(8, 8, 2, 2, wk.product_directions(4, 4), [3] * 4, seed=9, cfl=cfl)
        wl.integrator = "rk4"
        prob = dd.Problem(wl)
        h, om = prob.h, prob.omega[0]
        recs = []
        dd.stage_advect(dd.initial_state(wl), 0, prob, records=recs)
        es, el = [], []
        for rec in recs:
            U1, Vh, P, lam = rec["U1"], rec["V_hat"], rec["P"], rec["lam"]
            Kl, Kh = rec["Kb_lo"], rec["Kb_hi"]
            fS = lambda S: -(h * h) * (U1.T @ dd.kstep_rhs(U1 @ S, P, lam, Kl, Kh, 0, prob))
            es.append(rel(rec["S2"], _exact_affine_flow(fS, rec["S1"], prob.dt)))
            Gl, Gh = Kl @ Vh.T, Kh @ Vh.T
            fL = lambda L: ((h * h) * (U1.T @ dd.direction_rhs(U1 @ L.T, om, Gl, Gh, 0, prob))).T
            el.append(rel(rec["L1"], _exact_affine_flow(fL, Vh @ rec["S2"].T, prob.dt)))
        errs.append((max(es), max(el)))
    (s1, l1), (s2, l2) = errs
    assert 24.0 < s1 / s2 < 40.0 and 24.0 < l1 / l2 < 40.0, errs


def test_rk4_collision_substeps_local_error_is_fifth_order():
    """The collision K-, S- and L-step RK4 results (scattering, absorption
    and source all present) against the exact flows of the Euler right-hand
    sides (eqs. coll_evolK/S/L): halving dt divides the local error by about
    32."""
    errs = []
    for cfl in (0.2, 0.1):
        rng = np.random.default_rng(17)
        n = 64
        wl = wk.make_custom(8, 8, 2, 2, wk.product_directions(4, 4), [3, 4, 2, 3], seed=17, cfl=cfl,
                            sigma_s=rng.uniform(0.5, 3.0, n), sigma_a=rng.uniform(0.0, 2.0, n),
                            Q=rng.uniform(0.0, 1.0, n))
        wl.integrator = "rk4"
        prob = dd.Problem(wl)
        state = dd.initial_state(wl)
        recs = []
        dd.stage_collision(state, prob, records=recs)
        w, W, h, dt = prob.w, prob.W, prob.h, prob.dt
        ek, es, el = [], [], []
        for s, ((U, S, V), rec) in enumerate(zip(state, recs)):
            cs, ct, Qs, m = prob.sigma_s[s], prob.sigma_t[s], prob.Q[s], rec["m"]
            fK = lambda K: ((cs / W)[:, None] * (K @ m)[:, None] * m[None, :] - ct[:, None] * K
                            + Qs[:, None] * m[None, :])
            ek.append(rel(rec["K1"], _exact_affine_flow(fK, U @ S, dt)))
            Gs, Gt, q = rec["Gs"], rec["Gt"], rec["q"]
            fS = lambda X: -(1.0 / W) * Gs @ X @ np.outer(m, m) + Gt @ X - np.outer(q, m)
            es.append(rel(rec["S2"], _exact_affine_flow(fS, rec["S1"], dt)))
            ones = np.ones(prob.M)
            fL = lambda L: (1.0 / W) * np.outer(ones, (w @ L) @ Gs.T) - L @ Gt.T + np.outer(ones, q)
            el.append(rel(rec["L1"], _exact_affine_flow(fL, V @ rec["S2"].T, dt)))
        errs.append((max(ek), max(es), max(el)))
    for a, b in zip(errs[0], errs[1]):
        assert 24.0 < a / b < 40.0, errs
