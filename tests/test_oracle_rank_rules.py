"""Pins of the oracle's rank rules (Algorithm 4, step 3 and Algorithm 5,
step 2, with the caps of the readings R14/R15) and of the projector-splitting
exactness with exact sub-flows (Section 2: with exact flows of its substeps
the integrator reproduces the exact solution when the angular basis spans
every direction).

The expected ranks below are worked out by hand from the singular values
written in each test (tail sums of squares against the tolerance), not by
calling the rule: e.g. sigma = (1, 0.5, 0.1, 0.01, 0.001) and tol 0.02 give
tails sqrt(0.1^2 + 0.01^2 + 0.001^2) = 0.1005 after one value, 0.01005 after
two, so the tail rank is 2.
"""
import types

import numpy as np
import pytest
import scipy.linalg

import workloads as wk
from oracle import ddlra as dd
from oracle import sn_full as sn

from test_oracle_pins import SubGrid, full_rank_case, neighbour_inflow, rel, sub_block

SIG5 = np.array([1.0, 0.5, 0.1, 0.01, 0.001])   # tail rank 3 at tol 0.02, 4 at tol 0.005


def _prob(mode, r_fixed=3, r_min=1, r_max=8, r_int_max=16, tol=0.0, tol_aug_rel=1e-12):
    return types.SimpleNamespace(rank_mode=mode, r_fixed=r_fixed, r_min=r_min, r_max=r_max,
                                 r_int_max=r_int_max, tol=tol, tol_aug_rel=tol_aug_rel)


# ----------------------------------------------------------------------------
# Algorithm 4, step 3: t = max(r, tail rank), at most min(m0, r_int_max)
# ----------------------------------------------------------------------------

def test_aug_rank_tail_rule_adaptive():
    p = _prob(dd.RANK_ADAPTIVE, tol=0.02)
    assert dd.aug_rank(SIG5, 1, 5, p) == (3, False)
    # never below the current rank r
    assert dd.aug_rank(SIG5, 4, 5, p) == (4, False)
    p.tol = 0.005
    assert dd.aug_rank(SIG5, 1, 5, p) == (4, False)


def test_aug_rank_clamps_to_r_int_max_not_r_max():
    """The cap is r_int_max (the intermediate rank), not the stored-rank cap
    r_max; a clamp is reported."""
    p = _prob(dd.RANK_ADAPTIVE, tol=1e-9, r_max=2, r_int_max=4)
    assert dd.aug_rank(SIG5, 1, 5, p) == (4, True)     # tail rank 5, cap min(5, 4)
    p.r_int_max = 3
    assert dd.aug_rank(SIG5, 1, 5, p) == (3, True)


def test_aug_rank_clamps_to_m0():
    """With r_int_max above the augmented width m0 the cap is m0."""
    p = _prob(dd.RANK_ADAPTIVE, tol=1e-9, r_int_max=40)
    assert dd.aug_rank(SIG5, 1, 5, p) == (5, False)    # tail rank 5 = m0: no clamp
    sig = np.array([1.0, 0.5, 0.1])
    assert dd.aug_rank(sig, 1, 3, p) == (3, False)
    # a tolerance met at 5 with only 4 columns: the rule asks for 5
    sig6 = np.array([1.0, 0.5, 0.1, 0.01, 0.001, 1e-6])
    assert dd.aug_rank(sig6, 1, 4, p) == (4, True)


def test_aug_rank_fixed_mode_is_relative_to_sigma1():
    """Fixed-rank mode: the tolerance is tol_aug_rel * sigma_1."""
    p = _prob(dd.RANK_FIXED, tol_aug_rel=0.02, r_int_max=16)
    assert dd.aug_rank(10.0 * SIG5, 1, 5, p) == (3, False)   # tol 0.2 on sigma 10 * SIG5
    p.tol_aug_rel = 0.005
    assert dd.aug_rank(10.0 * SIG5, 1, 5, p) == (4, False)   # tol 0.05


def _aug_case(sig, r_int_max, tol):
    """One subdomain, no neighbours, L0 = V S^T with prescribed singular
    values (V weighted-orthonormal, S = diag(sig)): Algorithm 4 keeps the
    first t columns."""
    M = 12
    rng = np.random.default_rng(5)
    dirs = wk.paper_directions(M)
    w = dirs[2]
    k = len(sig)
    Q, _ = np.linalg.qr(rng.standard_normal((M, k)))
    V = Q / np.sqrt(w)[:, None]
    Uq, _ = np.linalg.qr(rng.standard_normal((16, k)))
    h = 0.25
    U = Uq / h
    S = np.diag(sig)
    prob = types.SimpleNamespace(w=w, h=h, rank_mode=dd.RANK_ADAPTIVE, r_fixed=k, r_min=1, r_max=k,
                                 r_int_max=r_int_max, tol=tol, tol_aug_rel=1e-12)
    return dd.augment(U, S, V, [], prob)


def test_augment_applies_the_rule_and_the_cap():
    K, Vh, t, sig, cl = _aug_case(SIG5, 16, 0.02)
    assert t == 5 and not cl and Vh.shape[1] == 5          # t >= r = 5 columns of S
    K, Vh, t, sig, cl = _aug_case(SIG5, 4, 0.02)
    assert t == 4 and cl and Vh.shape[1] == 4              # r = 5 > r_int_max = 4
    assert np.allclose(sig, SIG5, rtol=1e-12, atol=1e-15)


# ----------------------------------------------------------------------------
# Algorithm 5, step 2: r' = max(r_min, tail rank), at most min(r_max, t)
# ----------------------------------------------------------------------------

def test_trunc_rank_tail_rule():
    p = _prob(dd.RANK_ADAPTIVE, tol=0.02, r_min=1, r_max=8)
    assert dd.trunc_rank(SIG5, p) == (3, False)
    p.tol = 0.005
    assert dd.trunc_rank(SIG5, p) == (4, False)


def test_trunc_rank_respects_r_min():
    # tails: after 1 value sqrt(0.25+0.01+1e-4+1e-6) = 0.5101 > 0.5, after 2: 0.1005 -> tail rank 2
    p = _prob(dd.RANK_ADAPTIVE, tol=0.5, r_min=3, r_max=8)
    assert dd.trunc_rank(SIG5, p) == (3, False)
    p.r_min = 1
    assert dd.trunc_rank(SIG5, p) == (2, False)


def test_trunc_rank_clamps_to_r_max_and_reports():
    p = _prob(dd.RANK_ADAPTIVE, tol=1e-6, r_min=1, r_max=2)   # tail rank 5
    assert dd.trunc_rank(SIG5, p) == (2, True)
    p.r_max = 4
    assert dd.trunc_rank(SIG5, p) == (4, True)
    p.r_max = 9                                               # above t = 5: the cap is t
    assert dd.trunc_rank(SIG5, p) == (5, False)


def test_trunc_rank_fixed_mode():
    p = _prob(dd.RANK_FIXED, r_fixed=3, tol=1.0)
    assert dd.trunc_rank(SIG5, p) == (3, False)
    p.r_fixed = 7                                             # more than t columns
    assert dd.trunc_rank(SIG5, p) == (5, False)


def test_truncate_cuts_to_the_rule():
    rng = np.random.default_rng(8)
    Qa, _ = np.linalg.qr(rng.standard_normal((5, 5)))
    Qb, _ = np.linalg.qr(rng.standard_normal((5, 5)))
    S = Qa @ np.diag(SIG5) @ Qb.T
    U = np.eye(5)
    V = np.eye(5)
    p = _prob(dd.RANK_ADAPTIVE, tol=0.005, r_min=1, r_max=8)
    U1, S1, V1, sig, cl = dd.truncate(U, S, V, p)
    assert S1.shape == (4, 4) and not cl
    assert np.allclose(np.diag(S1), SIG5[:4], rtol=1e-13)
    # the discarded part is the tail
    assert abs(np.linalg.norm(S - U1 @ S1 @ V1.T) - 0.001) < 1e-14
    p.r_max = 2
    _, S2, _, _, cl2 = dd.truncate(U, S, V, p)
    assert S2.shape == (2, 2) and cl2


# ----------------------------------------------------------------------------
# exact sub-flows: full angular rank -> the exact frozen-inflow solution
# ----------------------------------------------------------------------------

def _exact(f, y0, dt):
    """exp flow of y' = f(y) (affine) from its dense matrix, by scipy expm."""
    shp = y0.shape
    n = y0.size
    b = f(np.zeros(shp)).ravel()
    A = np.column_stack([f(np.eye(n)[k].reshape(shp)).ravel() - b for k in range(n)])
    Z = np.zeros((n + 1, n + 1))
    Z[:n, :n] = A
    Z[:n, n] = b
    return (scipy.linalg.expm(dt * Z) @ np.append(y0.ravel(), 1.0))[:n].reshape(shp)


@pytest.mark.parametrize("axis", [0, 1])
def test_exact_subflows_full_rank_stage_is_exact(axis):
    """With exact sub-flows and full angular rank, the K-step reproduces the
    exact per-subdomain solution and the S-step (backward) and L-step
    (forward) flows cancel, so the whole stage output U1 S3 V1^T equals
    exp(dt A) F for the full-tensor upwind operator A of the subdomain with
    its inflow frozen at the start of the stage (SURVEY pin 3).  The Euler
    stage misses it at O(dt^2)."""
    wl = full_rank_case()
    prob = dd.Problem(wl)
    state = dd.initial_state(wl)
    F0 = sn.from_flat(dd.assemble(state, prob), wl)
    for integ, expect_exact in (("expm", True), ("euler", False)):
        wl.integrator = integ
        prob = dd.Problem(wl)
        recs = []
        dd.stage_advect(state, axis, prob, records=recs)
        for s, rec in enumerate(recs):
            g = SubGrid(wl, prob, s)
            lo, hi = neighbour_inflow(F0, prob, s, axis)
            Fs = sub_block(F0, prob, s).reshape(prob.lny, prob.lnx, -1)
            ref = _exact(lambda X: sn.advect_operator(X, axis, g, lo, hi), Fs, prob.dt).reshape(prob.N, -1)
            got = rec["U1"] @ rec["S3"] @ rec["V1"].T
            e = rel(got, ref)
            if expect_exact:
                assert e < 1e-12, (s, e)
            else:
                assert e > 1e-6, (s, e)


def test_exact_subflows_full_rank_collision_is_exact():
    """The collision stage with exact sub-flows at full angular rank equals
    exp(dt A_c) F with the full-tensor collision operator (scattering c_s rho
    / W, absorption, source) of each subdomain."""
    wl = full_rank_case(sigma=True)
    wl.integrator = "expm"
    prob = dd.Problem(wl)
    state = dd.initial_state(wl)
    out = dd.stage_collision(state, prob)
    F0 = sn.from_flat(dd.assemble(state, prob), wl)
    for s, (U1, S1, V1) in enumerate(out):
        g = SubGrid(wl, prob, s)
        Fs = sub_block(F0, prob, s).reshape(prob.lny, prob.lnx, -1)
        ref = _exact(lambda X: sn.collide_operator(X, g), Fs, prob.dt).reshape(prob.N, -1)
        assert rel(U1 @ S1 @ V1.T, ref) < 1e-12
