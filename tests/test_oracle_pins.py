"""Pins of the FP64 oracle against results the paper and the mathematics fix.

Nothing here compares the oracle with itself: each test checks it against an
independent computation (the full-tensor S_N scheme, a closed form, the
classic single-domain integrator, Eckart-Young, an exact shift).
"""
import math

import numpy as np
import pytest

import workloads as wk
from oracle import ddlra as dd
from oracle import psi_classic as pc
from oracle import sn_full as sn


# ----------------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------------

def full_rank_case(axis_dirs=False, seed=3, cfl=0.5, px=2, py=2, lnx=4, lny=4, M=8,
                   sigma=False):
    """Tiny problem where every subdomain holds F at full angular rank."""
    dirs = wk.axis_directions() if axis_dirs else wk.paper_directions(M)
    M = dirs[2].shape[0]
    nx, ny = px * lnx, py * lny
    ss = sa = Q = None
    if sigma:
        rng = np.random.default_rng(seed + 100)
        ss = rng.uniform(0.0, 2.0, nx * ny)
        sa = rng.uniform(0.0, 3.0, nx * ny)
        Q = rng.uniform(0.0, 1.0, nx * ny)
    return wk.make_custom(nx, ny, px, py, dirs, [M] * (px * py), seed=seed, cfl=cfl,
                          sigma_s=ss, sigma_a=sa, Q=Q, r_fixed=M, r_int_max=M,
                          sig=np.logspace(0, -1, M))


def sub_block(F3, prob, s):
    """F3[iy, ix, q] restricted to subdomain s in local order (N x M)."""
    sx, sy = s % prob.px, s // prob.px
    blk = F3[sy * prob.lny:(sy + 1) * prob.lny, sx * prob.lnx:(sx + 1) * prob.lnx, :]
    return blk.reshape(prob.N, -1)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def neighbour_inflow(F3, prob, s, axis):
    """Values of the global F in the cells just outside subdomain s along axis
    (zero at the physical boundary), shaped for sn_full's inflow arguments."""
    sx, sy = s % prob.px, s // prob.px
    ys = slice(sy * prob.lny, (sy + 1) * prob.lny)
    xs = slice(sx * prob.lnx, (sx + 1) * prob.lnx)
    M = F3.shape[2]
    if axis == 0:
        lo = F3[ys, sx * prob.lnx - 1, :] if sx > 0 else np.zeros((prob.lny, M))
        hi = F3[ys, (sx + 1) * prob.lnx, :] if sx < prob.px - 1 else np.zeros((prob.lny, M))
    else:
        lo = F3[sy * prob.lny - 1, xs, :] if sy > 0 else np.zeros((prob.lnx, M))
        hi = F3[(sy + 1) * prob.lny, xs, :] if sy < prob.py - 1 else np.zeros((prob.lnx, M))
    return lo, hi


class SubGrid:
    """sn_full grid restricted to one subdomain (same h, dt, directions)."""

    def __init__(self, wl, prob, s):
        cells = prob.local_cells(s)
        self.nx, self.ny, self.h = prob.lnx, prob.lny, prob.h
        self.ox, self.oy, self.w = prob.omega[0], prob.omega[1], prob.w
        self.W, self.c, self.dt = prob.W, prob.c, prob.dt
        self.ss = np.asarray(wl.sigma_s)[cells].reshape(prob.lny, prob.lnx)
        self.st = self.ss + np.asarray(wl.sigma_a)[cells].reshape(prob.lny, prob.lnx)
        self.Q = np.asarray(wl.Q)[cells].reshape(prob.lny, prob.lnx)


# ----------------------------------------------------------------------------
# quadrature (inputs shared by both sides)
# ----------------------------------------------------------------------------

def test_quadrature_weights_and_nodes():
    ox, oy, w = wk.product_directions(8, 8)
    assert abs(w.sum() - 4 * math.pi) < 1e-13
    assert np.allclose(ox ** 2 + oy ** 2 <= 1.0 + 1e-15, True)
    mu, wa = np.polynomial.legendre.leggauss(8)
    st = np.sqrt(1 - mu ** 2)
    assert np.allclose(np.sqrt(ox ** 2 + oy ** 2).reshape(8, 8)[:, 0], st)
    # first moments vanish, second moments are W/3 (isotropic)
    assert abs(np.sum(w * ox)) < 1e-13 and abs(np.sum(w * oy)) < 1e-13
    assert abs(np.sum(w * ox * ox) - 4 * math.pi / 3) < 1e-12
    ox, oy, w = wk.paper_directions(12)
    assert abs(w.sum() - 2 * math.pi) < 1e-14
    assert abs(np.sum(w * ox * ox) - math.pi) < 1e-13


def test_initial_factors_orthonormal():
    wl = wk.make_workload("C1")
    for U, S, V in zip(wl.U0, wl.S0, wl.V0):
        assert np.abs(wl.h ** 2 * U.T @ U - np.eye(U.shape[1])).max() < 1e-13
        assert np.abs(V.T @ (wl.w[:, None] * V) - np.eye(V.shape[1])).max() < 1e-13


# ----------------------------------------------------------------------------
# full angular rank: the K-step is the full-tensor upwind Euler step
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("axis", [0, 1])
def test_full_rank_kstep_equals_sn(axis):
    wl = full_rank_case()
    prob = dd.Problem(wl)
    state = dd.initial_state(wl)
    F0 = sn.from_flat(dd.assemble(state, prob), wl)
    g = sn.Grid(wl)
    F1 = sn.advect(F0, axis, g)
    recs = []
    dd.stage_advect(state, axis, prob, records=recs)
    for s, rec in enumerate(recs):
        assert rec["t"] == prob.M
        got = rec["K1"] @ rec["V_hat"].T
        assert rel(got, sub_block(F1, prob, s)) < 1e-12


def test_cfl_one_exact_shift():
    """c dt = h with directions on the axes: the x K-step moves every
    direction's profile by exactly one cell (textbook upwind)."""
    wl = full_rank_case(axis_dirs=True, cfl=1.0, lnx=5, lny=3)
    prob = dd.Problem(wl)
    state = dd.initial_state(wl)
    F0 = sn.from_flat(dd.assemble(state, prob), wl)
    exp = np.zeros_like(F0)
    exp[:, 1:, 0] = F0[:, :-1, 0]      # +x moves right, zero inflow
    exp[:, :-1, 2] = F0[:, 1:, 2]      # -x moves left
    exp[:, :, 1] = F0[:, :, 1]         # y directions untouched
    exp[:, :, 3] = F0[:, :, 3]
    recs = []
    dd.stage_advect(state, 0, prob, records=recs)
    for s, rec in enumerate(recs):
        got = rec["K1"] @ rec["V_hat"].T
        assert np.abs(got - sub_block(exp, prob, s)).max() < 1e-12 * np.abs(F0).max()


# ----------------------------------------------------------------------------
# full angular rank: closed form of one Euler PSI stage
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("axis", [0, 1])
def test_full_rank_advection_stage_closed_form(axis):
    wl = full_rank_case(seed=11)
    prob = dd.Problem(wl)
    state = dd.initial_state(wl)
    F0g = sn.from_flat(dd.assemble(state, prob), wl)
    F1g = sn.advect(F0g, axis, sn.Grid(wl))
    out = dd.stage_advect(state, axis, prob)
    for s in range(prob.n_sub):
        sg = SubGrid(wl, prob, s)
        lo, hi = neighbour_inflow(F0g, prob, s, axis)
        shape = (prob.lny, prob.lnx, prob.M)
        A = lambda X: sn.advect_operator(X.reshape(shape), axis, sg, lo, hi).reshape(prob.N, -1)  # noqa: E731
        A0 = lambda X: sn.advect_operator(X.reshape(shape), axis, sg).reshape(prob.N, -1)  # noqa: E731
        F1 = sub_block(F1g, prob, s)
        Uq, sv, _ = np.linalg.svd(F1, full_matrices=False)
        Q = Uq[:, : prob.M]
        PU = lambda X: Q @ (Q.T @ X)  # noqa: E731
        expect = F1 - prob.dt ** 2 * PU(A0(PU(A(F1))))
        U, S, V = out[s]
        got = U @ S @ V.T
        assert rel(got, expect) < 1e-12
        # and it is NOT the plain full-tensor step: the O(dt^2) term is real
        assert rel(got, F1) > 1e-6


def test_full_rank_collision_stage_closed_form():
    wl = full_rank_case(seed=5, sigma=True)
    prob = dd.Problem(wl)
    state = dd.initial_state(wl)
    out = dd.stage_collision(state, prob)
    for s in range(prob.n_sub):
        sg = SubGrid(wl, prob, s)
        U, S, V = state[s]
        F = U @ S @ V.T
        shape = (prob.lny, prob.lnx, prob.M)
        A = lambda X: sn.collide_operator(X.reshape(shape), sg).reshape(prob.N, -1)  # noqa: E731
        A0 = lambda X: sn.collide_operator(X.reshape(shape), sg, with_source=False).reshape(prob.N, -1)  # noqa: E731
        F1 = F + prob.dt * A(F)
        Uq, sv, _ = np.linalg.svd(F1, full_matrices=False)
        Q = Uq[:, : prob.M]
        PU = lambda X: Q @ (Q.T @ X)  # noqa: E731
        expect = F1 - prob.dt ** 2 * PU(A0(PU(A(F1))))
        U1, S1, V1 = out[s]
        assert rel(U1 @ S1 @ V1.T, expect) < 1e-12


def test_full_rank_whole_step_matches_sn_to_order_dt2():
    """Composition check: at full rank one DD step differs from the S_N step
    only by the O(dt^2) PSI terms, so halving dt divides the one-step
    difference by about 4."""
    errs = []
    for cfl in (0.2, 0.1):
        wl = full_rank_case(seed=9, cfl=cfl, sigma=True)
        prob = dd.Problem(wl)
        state = dd.initial_state(wl)
        F0 = sn.from_flat(dd.assemble(state, prob), wl)
        ref = sn.step(F0, sn.Grid(wl))
        got = dd.assemble(dd.dd_step(state, prob), prob)
        errs.append(rel(got, sn.to_flat(ref)))
    ratio = errs[0] / errs[1]
    assert 3.3 < ratio < 4.7, (errs, ratio)


# ----------------------------------------------------------------------------
# absorption, scattering, conservation
# ----------------------------------------------------------------------------

def _iso_init(N, M, r, h, w, rng, s):
    A = rng.standard_normal((N, r))
    B = np.hstack([np.ones((M, 1)), rng.standard_normal((M, r - 1))])
    return wk.factors_from_product(A, B, r, h, w)


def test_pure_absorption_factor():
    """c_s = 0, Q = 0, uniform sigma_a: the collision stage multiplies F by
    (1 - dt s)(1 + dt s)(1 - dt s) exactly (K-, S-, L-step), at any rank."""
    n = 8 * 8
    sa = 2.7
    wl = wk.make_custom(8, 8, 2, 2, wk.product_directions(4, 4), [3, 4, 2, 5], seed=2,
                        sigma_a=np.full(n, sa), cfl=0.5)
    prob = dd.Problem(wl)
    state = dd.initial_state(wl)
    out = dd.stage_collision(state, prob)
    fac = (1 - prob.dt * sa) * (1 + prob.dt * sa) * (1 - prob.dt * sa)
    for (U, S, V), (U1, S1, V1) in zip(state, out):
        assert rel(U1 @ S1 @ V1.T, fac * (U @ S @ V.T)) < 1e-14


def test_pure_absorption_converges_to_exponential():
    """Whole steps with c_adv = 0: F(T) -> exp(-sigma_a T) F(0), first order."""
    errs = []
    sa, T = 1.5, 0.4
    for nst in (8, 16, 32):
        wl = wk.make_custom(4, 4, 2, 2, wk.product_directions(4, 4), [2] * 4, seed=4,
                            sigma_a=np.full(16, sa), c_adv=0.0, r_int_max=6, r_fixed=2)
        wl.dt = T / nst
        prob = dd.Problem(wl)
        state = dd.initial_state(wl)
        F0 = dd.assemble(state, prob)
        for _ in range(nst):
            state = dd.dd_step(state, prob)
        errs.append(rel(dd.assemble(state, prob), math.exp(-sa * T) * F0))
    assert 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2, errs


def test_mass_conserved_under_pure_scattering():
    """c_adv = 0, sigma_a = 0, Q = 0, with the isotropic direction in span V:
    the total mass h^2 sum rho is conserved across K-, S- and L-steps."""
    n = 8 * 8
    rng = np.random.default_rng(8)
    wl = wk.make_custom(8, 8, 2, 2, wk.product_directions(4, 4), [3] * 4, seed=8,
                        sigma_s=rng.uniform(0.5, 4.0, n), c_adv=0.0, cfl=0.5,
                        r_int_max=9, init=_iso_init)
    wl.dt = 0.05
    prob = dd.Problem(wl)
    state = dd.initial_state(wl)
    m0 = prob.h ** 2 * dd.moments(state, prob).sum()
    for _ in range(5):
        state = dd.dd_step(state, prob)
    m1 = prob.h ** 2 * dd.moments(state, prob).sum()
    assert abs(m1 - m0) < 1e-13 * abs(m0)


def test_scattering_relaxes_to_isotropy():
    """Pure scattering at full angular rank keeps the mass of every cell and
    removes the anisotropic part at rate (1 - dt c_s) per K-step-dominated
    step; here only the cellwise mass check is exact."""
    wl = full_rank_case(seed=21)
    n = wl.nx * wl.ny
    wl.sigma_s = np.full(n, 3.0)
    wl.c_adv = 0.0
    prob = dd.Problem(wl)
    state = dd.initial_state(wl)
    rho0 = dd.moments(state, prob)
    out = dd.stage_collision(state, prob)
    assert rel(dd.moments(out, prob), rho0) < 1e-13


# ----------------------------------------------------------------------------
# domain decomposition specifics
# ----------------------------------------------------------------------------

def test_single_subdomain_equals_classic_split_psi():
    rng = np.random.default_rng(31)
    n = 6 * 5
    wl = wk.make_custom(6, 5, 1, 1, wk.product_directions(4, 4), [4], seed=31,
                        sigma_s=rng.uniform(0, 2, n), sigma_a=rng.uniform(0, 1, n),
                        Q=rng.uniform(0, 1, n), cfl=0.4)
    prob = dd.Problem(wl)
    state = dd.initial_state(wl)
    U, S, V = state[0]
    o = pc.Ops(wl)
    for _ in range(3):
        state = dd.dd_step(state, prob)
        U, S, V = pc.step(U, S, V, o)
    Ud, Sd, Vd = state[0]
    assert rel(Ud @ Sd @ Vd.T, U @ S @ V.T) < 1e-12


def test_random_augmentation_columns_have_no_effect():
    """Algorithm 4 with U_rand from two different seeds, and without it,
    gives the same stage result (the random columns meet a zero block)."""
    wl = wk.make_custom(8, 8, 2, 2, wk.product_directions(4, 4), [3, 2, 4, 3], seed=13, cfl=0.5)
    prob = dd.Problem(wl)
    state = dd.initial_state(wl)
    a = dd.stage_advect(state, 0, prob, rng=np.random.default_rng(1))
    b = dd.stage_advect(state, 0, prob, rng=np.random.default_rng(2))
    c = dd.stage_advect(state, 0, prob, rng=None)
    assert dd.state_rel_error(a, c, prob) < 1e-13
    assert dd.state_rel_error(b, c, prob) < 1e-13


def test_augmentation_projection_error_below_tail():
    """Eckart-Young for Algorithm 4: projecting F onto span(V-hat) loses at
    most the discarded tail of L^0's singular values."""
    wl = wk.make_custom(8, 8, 2, 2, wk.product_directions(6, 6), [4, 5, 3, 6], seed=17,
                        rank_mode=wk.RANK_ADAPTIVE, tol=3e-2, r_max=8, r_int_max=12,
                        sig=np.logspace(0, -3, 8))
    prob = dd.Problem(wl)
    state = dd.initial_state(wl)
    recs = []
    dd.stage_advect(state, 0, prob, records=recs)
    sw = np.sqrt(prob.w)
    for s, rec in enumerate(recs):
        U, S, V = state[s]
        t = rec["t"]
        tail = np.sqrt(np.sum(rec["sig_aug"][t:] ** 2))
        Vh = rec["V_hat"]
        L = V @ S.T
        err = np.linalg.norm(sw[:, None] * (L - Vh @ (Vh.T @ (prob.w[:, None] * L))))
        assert err <= tail * (1 + 1e-12) + 1e-15
        assert t >= U.shape[1]


def test_truncation_error_equals_tail():
    wl = wk.make_custom(4, 4, 1, 1, wk.product_directions(4, 4), [6], seed=19,
                        rank_mode=wk.RANK_ADAPTIVE, tol=0.05, r_max=6, r_int_max=6,
                        sig=np.logspace(0, -2, 6))
    prob = dd.Problem(wl)
    U, S, V = dd.initial_state(wl)[0]
    U1, S1, V1, sig, _ = dd.truncate(U, S, V, prob)
    rp = S1.shape[0]
    tail = np.sqrt(np.sum(sig[rp:] ** 2))
    assert tail <= 0.05 and np.sqrt(np.sum(sig[rp - 1:] ** 2)) > 0.05
    d = np.sqrt(max(dd.factored_dist2((U, S, V), (U1, S1, V1), prob), 0.0))
    assert abs(d - tail) < 1e-12


def test_full_rank_augmentation_is_noop():
    wl = full_rank_case(seed=23)
    prob = dd.Problem(wl)
    state = dd.initial_state(wl)
    recs = []
    dd.stage_advect(state, 0, prob, records=recs)
    for s, rec in enumerate(recs):
        U, S, V = state[s]
        assert rel(rec["K0"] @ rec["V_hat"].T, U @ S @ V.T) < 1e-13


def _mirror(wl, prob, axis):
    """Mirror image of a workload's initial factors: x -> -x (axis 0) or
    y -> -y (axis 1), with the matching permutation of the direction set."""
    n = prob.M
    phi = np.arctan2(prob.omega[1], prob.omega[0])
    mphi = (np.pi - phi) if axis == 0 else -phi
    perm = np.array([int(np.argmin(np.abs(np.angle(np.exp(1j * (phi - a)))))) for a in mphi])
    assert sorted(perm.tolist()) == list(range(n))
    U0, S0, V0 = [None] * prob.n_sub, [None] * prob.n_sub, [None] * prob.n_sub
    loc = np.arange(prob.N).reshape(prob.lny, prob.lnx)
    loc = loc[:, ::-1] if axis == 0 else loc[::-1, :]
    for s in range(prob.n_sub):
        sx, sy = s % prob.px, s // prob.px
        t = (sy * prob.px + (prob.px - 1 - sx)) if axis == 0 else ((prob.py - 1 - sy) * prob.px + sx)
        U0[t] = wl.U0[s][loc.ravel()]
        S0[t] = wl.S0[s]
        V0[t] = wl.V0[s][perm]
    return U0, S0, V0, loc.ravel(), perm


@pytest.mark.parametrize("axis", [0, 1])
def test_mirror_symmetry_low_rank(axis):
    """Reflecting the grid and the direction set commutes with a whole DD
    step at low rank: a left/right (or bottom/top) mix-up in the inflow
    transfer, the faces or the upwind sides breaks this."""
    rng = np.random.default_rng(43)
    nx, ny, px, py = 12, 8, 3, 2
    n = nx * ny
    ss = rng.uniform(0, 2, (ny, nx))
    sa = rng.uniform(0, 1, (ny, nx))
    Q = rng.uniform(0, 1, (ny, nx))
    ss = ss + (ss[:, ::-1] if axis == 0 else ss[::-1, :])
    sa = sa + (sa[:, ::-1] if axis == 0 else sa[::-1, :])
    Q = Q + (Q[:, ::-1] if axis == 0 else Q[::-1, :])
    wl = wk.make_custom(nx, ny, px, py, wk.paper_directions(12), [3, 4, 2, 3, 5, 2], seed=43,
                        sigma_s=ss.ravel(), sigma_a=sa.ravel(), Q=Q.ravel(), cfl=0.4,
                        rank_mode=wk.RANK_ADAPTIVE, tol=1e-3, r_max=6, r_int_max=10)
    prob = dd.Problem(wl)
    U0, S0, V0, loc, perm = _mirror(wl, prob, axis)
    wm = wl.with_factors(U0, S0, V0)
    a = dd.dd_step(dd.initial_state(wl), prob)
    b = dd.dd_step(dd.initial_state(wm), prob)
    Fa = dd.assemble(a, prob).reshape(ny, nx, -1)
    Fb = dd.assemble(b, prob).reshape(ny, nx, -1)
    Fa_m = (Fa[:, ::-1, :] if axis == 0 else Fa[::-1, :, :])[:, :, perm]
    assert rel(Fb, Fa_m) < 1e-12


# ----------------------------------------------------------------------------
# observables: current density (first angular moments)
# ----------------------------------------------------------------------------

def test_currents_equal_assembled_distribution():
    """jx, jy from the factors equal the quadrature of Omega f over the
    assembled full distribution (brute force on the C1 grid)."""
    wl = wk.make_workload("wc-C1")
    prob = dd.Problem(wl)
    state = dd.initial_state(wl)
    F = dd.assemble(state, prob)
    jx, jy = dd.currents(state, prob)
    assert rel(jx, F @ (prob.w * prob.omega[0])) < 1e-13
    assert rel(jy, F @ (prob.w * prob.omega[1])) < 1e-13
    assert rel(dd.moments(state, prob), F @ prob.w) < 1e-13


def test_isotropic_distribution_carries_no_current():
    """An isotropic f(x, Omega) = g(x) has zero current: the direction set is
    symmetric, so sum_q w_q Omega_q = 0."""
    wl = wk.make_workload("wc-C1")
    prob = dd.Problem(wl)
    rng = np.random.default_rng(11)
    state = []
    for s in range(prob.n_sub):
        g = rng.standard_normal(prob.N)
        U = (g / (prob.h * np.linalg.norm(g)))[:, None]          # h^2 U^T U = 1
        V = np.full((prob.M, 1), 1.0 / math.sqrt(prob.W))        # V^T W V = 1
        state.append((U, np.array([[2.0]]), V))
    rho = dd.moments(state, prob)
    jx, jy = dd.currents(state, prob)
    scale = np.linalg.norm(rho)
    assert np.linalg.norm(jx) < 1e-14 * scale and np.linalg.norm(jy) < 1e-14 * scale
