"""RK4 substeps in the engine against the oracle's classic four-stage
Runge-Kutta substeps (boundary data frozen over each substep).

The engine evaluates each affine substep in the nested form
y1 = y0 + dt f(y0 + dt/2 f(y0 + dt/3 f(y0 + dt/4 f(y0)))) or through the
equivalent degree-4 Taylor polynomial, which equal the classic RK4 step up to
rounding for an affine autonomous f; the bar is the FP64 one (1e-10).
"""
import dataclasses

import numpy as np
import pytest

import workloads as wk
from oracle import ddlra as dd

from test_gpu_parity import STRICT, engine, rho_err, say
from test_gpu_wide import graded_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_14854_amd as pkg
    pkg.load_library()


def rk4(wl):
    return dataclasses.replace(wl, integrator="rk4")


@pytest.mark.parametrize("stage", [0, 1, 2])
def test_rk4_single_stages(stage):
    """Each stage of wc-C1 with RK4 substeps: x advection, y advection,
    collision."""
    wl = rk4(wk.make_workload("wc-C1"))
    say(f"case: wc-C1 with RK4 substeps, stage {stage}")
    prob = dd.Problem(wl)
    st0 = dd.initial_state(wl)
    ref = dd.stage_advect(st0, stage, prob) if stage < 2 else dd.stage_collision(st0, prob)
    e = engine(wl)
    e.stage(stage)
    got = e.state()
    e.close()
    err = dd.state_rel_error(got, ref, prob)
    say(f"  state err {err:.3e}")
    assert err < STRICT


@pytest.mark.parametrize("name,nsteps", [("wc-C1", 2), ("wc-C2", 2)])
def test_rk4_steps(name, nsteps):
    """Whole steps with RK4 substeps: state and scalar flux within 1e-10 of
    the oracle, and visibly different from the Euler substeps (the path is
    the RK4 one)."""
    wl = rk4(wk.make_workload(name))
    say(f"case: {name} with RK4 substeps, {nsteps} steps")
    prob = dd.Problem(wl)
    st = dd.initial_state(wl)
    for _ in range(nsteps):
        st = dd.dd_step(st, prob)
    e = engine(wl)
    e.step(nsteps)
    got = e.state()
    rho = e.moments()
    e.close()
    e = engine(dataclasses.replace(wl, integrator="euler"))
    e.step(nsteps)
    rho_euler = e.moments()
    e.close()
    ref_rho = dd.moments(st, prob)
    err, ferr = dd.state_rel_error(got, st, prob), rho_err(rho, ref_rho)
    gap = rho_err(rho_euler, ref_rho)
    say(f"  state err {err:.3e}, flux err {ferr:.3e}; Euler substeps differ by {gap:.3e}")
    assert err < STRICT and ferr < STRICT
    assert gap > 1e3 * max(ferr, 1e-15)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("stage", [0, 1, 2])
def test_rk4_wide_ranks(stage):
    """RK4 substeps at intermediate ranks up to 128 (2x2 of 16x16 cells,
    256 directions, ranks 20..32, adaptive)."""
    wl = rk4(graded_case([20, 24, 28, 32]))
    say(f"case: 2x2 of 16x16, M=256, ranks 20..32, RK4 substeps, stage {stage}")
    prob = dd.Problem(wl)
    st0 = dd.initial_state(wl)
    recs = []
    if stage < 2:
        ref = dd.stage_advect(st0, stage, prob, records=recs)
    else:
        ref = dd.stage_collision(st0, prob)
    e = engine(wl)
    e.stage(stage)
    got = e.state()
    r, tmax, _ = e.ranks()
    e.close()
    err = dd.state_rel_error(got, ref, prob)
    say(f"  state err {err:.3e}, ranks {list(r)}, t {list(tmax)}")
    if recs:
        assert list(tmax) == [x["t"] for x in recs]
    assert list(r) == [S.shape[0] for _, S, _ in ref]
    assert err < 1e-11


def test_rk4_exec_modes_bitwise_equal():
    import paper_2602_14854_amd as pkg
    wl = rk4(wk.make_workload("wc-C1"))
    say("case: wc-C1 RK4, exec modes")
    out = []
    for mode in (pkg.DD_EXEC_PER_SUBDOMAIN, pkg.DD_EXEC_BATCHED, pkg.DD_EXEC_BATCHED_GRAPH):
        e = engine(wl, exec_mode=mode)
        e.step(2)
        out.append(e.state())
        e.close()
    for other in out[1:]:
        for a, b in zip(out[0], other):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)
