"""Pins of the oracle's physical inflow faces (prescribed inflow of the
paper's Hohlraum and boundary point-source problems, Section 4) against the
full-tensor S_N scheme and an exact steady state."""
import numpy as np
import pytest

import workloads as wk
from oracle import ddlra as dd
from oracle import sn_full as sn

from test_oracle_pins import full_rank_case, sub_block, rel


def _inflow_case(axis, seed=3):
    """2x2 subdomains of 4x4 cells at full angular rank (M = 8), a rank-2
    random inflow on the low face of the given axis, vacuum elsewhere."""
    wl = full_rank_case(seed=seed)
    rng = np.random.default_rng(seed + 50)
    n_face = wl.ny if axis == 0 else wl.nx
    A = rng.standard_normal((n_face, 2))
    B = rng.standard_normal((wl.w.shape[0], 2))
    inflow = [None] * 4
    inflow[0 if axis == 0 else 2] = (A, B)
    wl.inflow = inflow
    return wl, A, B


@pytest.mark.parametrize("axis", [0, 1])
def test_full_rank_kstep_with_inflow_equals_sn(axis):
    """At full angular rank the K-step of a stage with a prescribed inflow on
    the physical low face is the S_N upwind step with that inflow in the
    ghost cells (1e-12): the inflow reaches the directions entering through
    the face, at the right cells."""
    wl, A, B = _inflow_case(axis)
    prob = dd.Problem(wl)
    state = dd.initial_state(wl)
    F0 = sn.from_flat(dd.assemble(state, prob), wl)
    g = sn.Grid(wl)
    F1 = sn.advect(F0, axis, g, inflow_lo=A @ B.T)
    recs = []
    dd.stage_advect(state, axis, prob, records=recs)
    for s, rec in enumerate(recs):
        assert rec["t"] == prob.M
        got = rec["K1"] @ rec["V_hat"].T
        assert rel(got, sub_block(F1, prob, s)) < 1e-12


def test_inflow_layer_reproduces_the_prescribed_values():
    """The layer's factors U_v S_v V_v^T equal the prescribed inflow A B^T on
    the layer's cells next to each boundary subdomain, and the interior
    faces have no layer."""
    wl, A, B = _inflow_case(0)
    prob = dd.Problem(wl)
    for s in range(prob.n_sub):
        v = prob.virtual_neighbour(s, 0, -1)
        if s % prob.px != 0:
            assert v is None
            continue
        U, S, V = v
        sy = s // prob.px
        rows = U[prob.face(0, True)] @ S @ V.T
        assert rel(rows, A[sy * prob.lny:(sy + 1) * prob.lny] @ B.T) < 1e-13
        assert prob.virtual_neighbour(s, 0, +1) is None   # vacuum on +x


def test_constant_inflow_reaches_the_exact_steady_state():
    """Pure advection along the axes (4 directions), zero initial state,
    f_in = 1 for the +x direction on the -x face, vacuum elsewhere, adaptive
    ranks capped below the angular dimension (r_max 2 < M = 4).  The upwind
    steady state is f = 1 in the +x direction everywhere and 0 otherwise
    (rank 1); the DD step reaches it to 1e-12 after the front has crossed
    the grid.  The initial basis cannot represent the +x direction, so the
    inflow must enter through the augmentation (R33)."""
    dirs = wk.axis_directions()
    M = 4
    nx = ny = 8
    z = lambda N, M_, r, h, w, rng, s: (np.linalg.qr(rng.standard_normal((N, 1)))[0] / h,
                                        np.zeros((1, 1)),
                                        (np.linalg.qr(np.sqrt(w)[:, None] * rng.standard_normal((M_, 1)))[0]
                                         / np.sqrt(w)[:, None]))
    wl = wk.make_custom(nx, ny, 2, 2, dirs, [1] * 4, seed=5, cfl=0.5, rank_mode=wk.RANK_ADAPTIVE,
                        tol=1e-13, r_max=2, r_int_max=4, r_min=1, init=z)
    B = np.array([[1.0], [0.0], [0.0], [0.0]])
    wl.inflow = [(np.ones((ny, 1)), B), None, None, None]
    prob = dd.Problem(wl)
    st = dd.initial_state(wl)
    for _ in range(200):
        st = dd.dd_step(st, prob)
    F = dd.assemble(st, prob)
    exp = np.zeros((nx * ny, M))
    exp[:, 0] = 1.0
    assert np.abs(F - exp).max() < 1e-12
    assert max(S.shape[0] for _, S, _ in st) <= 2


def test_augmentation_takes_the_inflow_profile():
    """From a zero state (rank 1, S = 0) the x stage's augmentation of a
    subdomain on an inflow face has L0 = [0, h B R_a^T] (and a neighbour's
    zero block): its one nonzero singular value is h ||a_s|| ||B||_w and
    V-hat (t = 1) is the inflow's angular profile B; elsewhere L0 is zero
    (R33)."""
    dirs = wk.paper_directions(8)
    nx = ny = 8
    rng = np.random.default_rng(9)

    def zero(N, M_, r, h, w, rng_, s):
        U = np.linalg.qr(rng_.standard_normal((N, 1)))[0] / h
        V = np.linalg.qr(np.sqrt(w)[:, None] * rng_.standard_normal((M_, 1)))[0] / np.sqrt(w)[:, None]
        return U, np.zeros((1, 1)), V

    wl = wk.make_custom(nx, ny, 2, 2, dirs, [1] * 4, seed=6, cfl=0.5, rank_mode=wk.RANK_ADAPTIVE,
                        tol=1e-10, r_max=4, r_int_max=8, r_min=1, init=zero)
    a = rng.uniform(0.5, 1.5, (ny, 1))
    B = rng.uniform(0.0, 1.0, (8, 1)) * (dirs[0][:, None] >= 0)
    wl.inflow = [(a, B), None, None, None]
    prob = dd.Problem(wl)
    recs = []
    dd.stage_advect(dd.initial_state(wl), 0, prob, records=recs)
    w = prob.w
    for s, rec in enumerate(recs):
        if s % prob.px == 0:
            sy = s // prob.px
            a_s = a[sy * prob.lny:(sy + 1) * prob.lny, 0]
            expect = prob.h * np.linalg.norm(a_s) * np.sqrt(np.sum(w * B[:, 0] ** 2))
            assert rec["t"] == 1
            assert abs(rec["sig_aug"][0] - expect) < 1e-12 * expect
            assert np.all(rec["sig_aug"][1:] < 1e-14 * expect)
            Vh = rec["V_hat"]
            proj = Vh @ (Vh.T @ (w * B[:, 0]))
            assert np.linalg.norm(np.sqrt(w) * (B[:, 0] - proj)) < 1e-12 * np.linalg.norm(np.sqrt(w) * B[:, 0])
        else:
            assert rec["t"] == 1 and np.all(rec["sig_aug"] == 0.0)
