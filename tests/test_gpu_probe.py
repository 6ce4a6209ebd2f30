"""Phase-by-phase parity of an advection stage (Algorithm 4's augmentation,
then the K-, QR-, S- and L-steps of Algorithms 1/2) through the stage
probe of the C ABI, against the intermediate results the FP64 oracle records.

The bases are not unique, so each phase is compared through a product that
does not depend on them: the projector onto V-hat, K1 V-hat^T, the projector
onto U1, U1 S2 V-hat^T and U1 L1^T (the distribution after the K-, S- and
L-steps).  A failure names the first phase that departs from the oracle.
The projector onto U1 moves by about u * cond(K1) when K1 is perturbed by
u relative (u the unit roundoff of the stored K1), so its bar is the larger
of the case's bar and 10 u cond(K1).
"""
import dataclasses

import numpy as np
import pytest

import workloads as wk
from oracle import ddlra as dd

from test_gpu_parity import engine, say, small_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_14854_amd as pkg
    pkg.load_library()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def phase_errors(e, wl, stage, subdomains=None):
    """Relative errors of the five phases of stage `stage` for each
    subdomain, the engine's t against the oracle's, and that the probes left
    the state untouched."""
    import paper_2602_14854_amd as pkg
    prob = dd.Problem(wl)
    st0 = dd.initial_state(wl)
    recs = []
    dd.stage_advect(st0, stage, prob, records=recs)
    sw = np.sqrt(prob.w)[:, None]
    before = e.state()
    out = []
    for s in (subdomains if subdomains is not None else range(prob.n_sub)):
        rec = recs[s]
        Qh = e.probe(stage, pkg.DD_PROBE_VHAT, s)
        K1 = e.probe(stage, pkg.DD_PROBE_K1, s)
        hU1 = e.probe(stage, pkg.DD_PROBE_U1, s)
        S2 = e.probe(stage, pkg.DD_PROBE_S2, s)
        AL = e.probe(stage, pkg.DD_PROBE_L1, s)
        t = Qh.shape[1]
        assert t == rec["t"], (s, t, rec["t"])
        assert K1.shape == (prob.N, t) and hU1.shape == (prob.N, t)
        assert S2.shape == (t, t) and AL.shape == (prob.M, t)
        Vh = Qh / sw                       # V-hat, V^T W V = I
        U1 = hU1 / prob.h                  # h^2 U^T U = I
        L1 = AL / sw
        QhO = sw * rec["V_hat"]
        hU1O = prob.h * rec["U1"]
        errs = {
            "vhat": rel(Qh @ Qh.T, QhO @ QhO.T),
            "k1": rel(K1 @ Vh.T, rec["K1"] @ rec["V_hat"].T),
            "u1": rel(hU1 @ hU1.T, hU1O @ hU1O.T),
            "s2": rel(U1 @ S2 @ Vh.T, rec["U1"] @ rec["S2"] @ rec["V_hat"].T),
            "l1": rel(U1 @ L1.T, rec["U1"] @ rec["L1"].T),
            "cond_k1": float(np.linalg.cond(rec["K1"])),
        }
        out.append((s, errs))
    after = e.state()
    for a, b in zip(before, after):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    return out


def check(e, wl, stage, bar, label, subdomains=None, unit=2.0 ** -53):
    worst = {}
    for s, errs in phase_errors(e, wl, stage, subdomains):
        for k, v in errs.items():
            if k != "cond_k1":
                worst[k] = max(worst.get(k, 0.0), v)
        assert errs["u1"] < max(bar, 10 * unit * errs["cond_k1"]), (s, errs)
    say(f"  {label} stage {stage}: " + ", ".join(f"{k} {v:.2e}" for k, v in worst.items()))
    for k in ("vhat", "k1", "s2", "l1"):
        assert worst[k] < bar, (k, worst[k])


@pytest.mark.parametrize("stage", [0, 1])
def test_probe_phases_narrow_wc_C1(stage):
    wl = wk.make_workload("wc-C1")
    say(f"case: wc-C1 (32x32, 2x2, M=64, r=5), narrow plan, stage {stage}, all phases")
    e = engine(wl)
    check(e, wl, stage, 1e-12, "narrow")
    e.close()


@pytest.mark.parametrize("stage", [0, 1])
def test_probe_phases_wide_wc_C1(stage, monkeypatch):
    monkeypatch.setenv("DD_DLRA_PLAN", "wide")
    wl = wk.make_workload("wc-C1")
    say(f"case: wc-C1, wide plan, stage {stage}, all phases")
    e = engine(wl)
    check(e, wl, stage, 1e-12, "wide")
    e.close()


@pytest.mark.timeout(300)
def test_probe_phases_wide_medium_ranks():
    """Ranks 20 to 32 with 256 directions (the wide plan by capacity), factors
    graded 1 ... 1e-4, adaptive."""
    from test_gpu_wide import graded_case
    wl = graded_case([20, 24, 28, 32])
    say("case: 2x2 of 16x16, M=256, ranks 20..32, x stage, all phases")
    e = engine(wl)
    check(e, wl, 0, 1e-11, "wide medium")
    e.close()


def test_probe_phases_rk4():
    wl = dataclasses.replace(small_case(seed=6), integrator="rk4")
    say("case: 2x2 of 8x8, M=16, r=3, RK4 substeps, both stages, all phases")
    e = engine(wl)
    for stage in (0, 1):
        check(e, wl, stage, 1e-12, "rk4")
    e.close()


def test_probe_phases_mixed_fp32():
    """FP32 storage of V-hat, K1 and L1: every phase within 1e-5 (the U1
    projector within 10 u cond(K1), u = 2^-24)."""
    import paper_2602_14854_amd as pkg
    wl = wk.make_workload("wc-C1")
    say("case: wc-C1, narrow plan, mixed FP32, x stage, all phases")
    e = engine(wl, precision=pkg.DD_PREC_MIXED_FP32)
    check(e, wl, 0, 1e-5, "mixed fp32", unit=2.0 ** -24)
    e.close()


def test_probe_then_step_is_unchanged():
    """Probing before a step changes nothing the step computes (bitwise)."""
    import paper_2602_14854_amd as pkg
    wl = small_case(seed=8)
    e1 = engine(wl)
    for stage in (0, 1):
        for upto in (pkg.DD_PROBE_VHAT, pkg.DD_PROBE_S2, pkg.DD_PROBE_L1):
            e1.probe(stage, upto, 1)
    e1.step(2)
    a = e1.state()
    e1.close()
    e2 = engine(wl)
    e2.step(2)
    b = e2.state()
    e2.close()
    for fa, fb in zip(a, b):
        for x, y in zip(fa, fb):
            assert np.array_equal(x, y)


def test_probe_arguments_validated():
    import paper_2602_14854_amd as pkg
    from paper_2602_14854_amd import DDError
    wl = small_case(seed=8)
    e = engine(wl)
    for args in ((2, pkg.DD_PROBE_K1, 0), (0, 0, 0), (0, 6, 0), (0, pkg.DD_PROBE_K1, 4), (0, pkg.DD_PROBE_K1, -1)):
        with pytest.raises(DDError):
            e.probe(*args)
    e.close()
