"""Physical inflow faces (prescribed low-rank inflow, the paper's Hohlraum
and boundary point-source problems of Section 4) through the C ABI against
the FP64 oracle, in both launch plans."""
import dataclasses
import math

import numpy as np
import pytest

import workloads as wk
from oracle import ddlra as dd

from test_gpu_parity import STRICT, engine, rho_err, say, small_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_14854_amd as pkg
    pkg.load_library()


def hohlraum_like(px=2, py=2, lnx=8, adaptive=False, seed=5, **kw):
    """f_in = 1 on the -x face for the directions entering it (Omega_x >= 0),
    a random rank-2 inflow on the +y face, vacuum on the other two."""
    dirs = wk.product_directions(4, 4)
    args = dict(seed=seed, px=px, py=py, lnx=lnx, lny=lnx, dirs=dirs, ranks=[3] * (px * py))
    if adaptive:
        args.update(rank_mode=wk.RANK_ADAPTIVE, tol=1e-6, r_max=6, r_int_max=12, r_min=1)
    args.update(kw)
    wl = small_case(**args)
    rng = np.random.default_rng(seed + 7)
    B0 = (np.asarray(wl.omega_x) >= 0).astype(float)[:, None]
    A2 = rng.uniform(0.0, 1.0, (wl.nx, 2))
    B2 = rng.uniform(0.0, 1.0, (wl.w.shape[0], 2)) * (np.asarray(wl.omega_y) < 0)[:, None]
    wl.inflow = [(np.ones((wl.ny, 1)), B0), None, None, (A2, B2)]
    return wl


def boundary_point_source(px=3, py=3, lnx=8, seed=9):
    """A narrow Gaussian inflow profile near the top of the -x face, the
    directions entering it, adaptive ranks (Section 4's boundary point
    source, at a small size)."""
    dirs = wk.product_directions(4, 6)
    wl = small_case(seed=seed, px=px, py=py, lnx=lnx, lny=lnx, dirs=dirs, ranks=[2] * (px * py),
                    rank_mode=wk.RANK_ADAPTIVE, tol=1e-8, r_max=8, r_int_max=16, r_min=1)
    h = (wl.x1 - wl.x0) / wl.nx
    y = (np.arange(wl.ny) + 0.5) * h
    sig = 2.0 * h
    g = np.exp(-(y - 0.85 * wl.ny * h) ** 2 / (2 * sig * sig)) / (math.sqrt(2 * math.pi) * sig)
    B = (np.asarray(wl.omega_x) >= 0).astype(float)[:, None]
    wl.inflow = [(g[:, None], B), None, None, None]
    return wl


def compare(wl, nsteps, label, monkeypatch=None, bar=STRICT):
    prob = dd.Problem(wl)
    st = dd.initial_state(wl)
    for _ in range(nsteps):
        st = dd.dd_step(st, prob)
    e = engine(wl)
    e.step(nsteps)
    got = e.state()
    rho = e.moments()
    r, _, _ = e.ranks()
    e.close()
    err, ferr = dd.state_rel_error(got, st, prob), rho_err(rho, dd.moments(st, prob))
    say(f"  {label}: state err {err:.3e}, flux err {ferr:.3e}, ranks {list(r)}")
    assert list(r) == [S.shape[0] for _, S, _ in st]
    assert err < bar and ferr < bar
    return rho


@pytest.mark.parametrize("plan", ["narrow", "wide"])
def test_inflow_faces_fixed_rank(plan, monkeypatch):
    if plan == "wide":
        monkeypatch.setenv("DD_DLRA_PLAN", "wide")
    wl = hohlraum_like()
    say(f"case: 2x2 of 8x8, M=16, rank 3, inflow on -x (uniform) and +y (rank 2), {plan} plan, 3 steps")
    compare(wl, 3, plan)


@pytest.mark.parametrize("plan", ["narrow", "wide"])
def test_inflow_faces_adaptive(plan, monkeypatch):
    """Adaptive ranks: the inflow's angular profile enters through the
    augmentation, so the boundary subdomains grow their ranks."""
    if plan == "wide":
        monkeypatch.setenv("DD_DLRA_PLAN", "wide")
    wl = hohlraum_like(adaptive=True)
    say(f"case: 2x2 of 8x8, adaptive, inflow on -x and +y, {plan} plan, 4 steps")
    compare(wl, 4, plan)


def test_boundary_point_source():
    wl = boundary_point_source()
    say("case: 3x3 of 8x8, M=24, adaptive, Gaussian inflow near the top of -x, 6 steps")
    rho = compare(wl, 6, "point source")
    assert np.max(rho) > 0.0


def test_inflow_with_rk4_substeps():
    wl = dataclasses.replace(hohlraum_like(adaptive=True), integrator="rk4")
    say("case: 2x2 of 8x8, adaptive, inflow on -x and +y, RK4 substeps, 3 steps")
    compare(wl, 3, "rk4")


def test_inflow_exec_modes_bitwise_equal():
    import paper_2602_14854_amd as pkg
    wl = hohlraum_like(adaptive=True)
    out = []
    for mode in (pkg.DD_EXEC_PER_SUBDOMAIN, pkg.DD_EXEC_BATCHED, pkg.DD_EXEC_BATCHED_GRAPH):
        e = engine(wl, exec_mode=mode)
        e.step(3)
        out.append(e.state())
        e.close()
    for other in out[1:]:
        for a, b in zip(out[0], other):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)
