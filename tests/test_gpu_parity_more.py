"""More parity checks of the HIP path (through the C ABI) against the FP64
oracle: the moments cell by cell, the distance and the singular values of
every subdomain, directions along the axes (Omega_x = 0 or Omega_y = 0
exactly), ranks imposed through dd_dlra_force_ranks against the oracle with
the same ranks imposed, and the rank-capacity clamps (counted, or latched as
DD_ERANK in strict mode)."""
import math

import numpy as np
import pytest

import workloads as wk
from oracle import ddlra as dd

from test_gpu_parity import STRICT, engine, say, small_case, oracle_steps

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_14854_amd as pkg
    pkg.load_library()


def per_subdomain(got, ref, prob):
    """(largest distance of a subdomain relative to its own norm, or to 1e-3
    of the largest subdomain norm if that is more; largest singular-value
    difference relative to the subdomain's largest singular value; ranks
    equal)."""
    norms = [float(np.linalg.norm(S)) for _, S, _ in ref]
    big = max(norms)
    dist, sdiff = 0.0, 0.0
    for s in range(len(ref)):
        d2 = max(dd.factored_dist2(got[s], ref[s], prob), 0.0)
        dist = max(dist, math.sqrt(d2) / max(norms[s], 1e-3 * big))
        sg = np.linalg.svd(got[s][1], compute_uv=False)
        sr = np.linalg.svd(ref[s][1], compute_uv=False)
        assert sg.shape == sr.shape, f"subdomain {s}: rank {sg.size} against {sr.size}"
        if sr.size and sr[0] > 0:
            sdiff = max(sdiff, float(np.max(np.abs(sg - sr))) / sr[0])
    return dist, sdiff


def maxnorm(a, b, scale):
    return float(np.max(np.abs(a - b)) / scale)


def test_cellwise_moments_and_per_subdomain_state():
    """wc-C1, two steps: every subdomain within 1e-10 of the oracle (factored
    distance and singular values), and the scalar flux and both current
    densities cell by cell within 1e-10 of the largest flux value."""
    wl = wk.make_workload("wc-C1")
    say("case: wc-C1, 2 steps, cell by cell and subdomain by subdomain")
    ref, prob = oracle_steps(wl, 2)
    e = engine(wl)
    e.step(2)
    got = e.state()
    rho, jx, jy = e.currents()
    e.close()
    dist, sdiff = per_subdomain(got, ref, prob)
    rr = dd.moments(ref, prob)
    rx, ry = dd.currents(ref, prob)
    scale = float(np.max(np.abs(rr)))
    m = [maxnorm(rho, rr, scale), maxnorm(jx, rx, scale), maxnorm(jy, ry, scale)]
    say(f"  subdomain distance {dist:.3e}, singular values {sdiff:.3e}, max-norm rho/jx/jy "
        f"{m[0]:.3e} {m[1]:.3e} {m[2]:.3e}")
    assert dist < STRICT and sdiff < STRICT
    assert max(m) < STRICT


def axis_directions_8():
    """Eight directions at multiples of 45 degrees, components exactly 0 on
    the axes, weights 2 pi / 8."""
    phi = np.arange(8) * (2.0 * math.pi / 8)
    ox, oy = np.cos(phi), np.sin(phi)
    ox[np.abs(ox) < 1e-12] = 0.0
    oy[np.abs(oy) < 1e-12] = 0.0
    return ox, oy, np.full(8, 2.0 * math.pi / 8)


def test_directions_along_the_axes():
    """Directions with Omega_x = 0 or Omega_y = 0 exactly, at full angular
    rank (t = M = 8): the matrix C of each advection stage then has exact
    zero eigenvalues (up to rounding), the sign-function split meets them,
    and the upwind classes of the L-step meet Omega = 0.  Two steps match
    the oracle subdomain by subdomain."""
    dirs = axis_directions_8()
    wl = small_case(seed=17, px=2, py=2, lnx=8, lny=8, dirs=dirs, ranks=[8] * 4, r_fixed=8, r_int_max=8,
                    sig=np.logspace(0, -2, 8))
    say("case: 2x2 of 8x8, 8 directions on the axes and diagonals, full rank 8")
    ref, prob = oracle_steps(wl, 2)
    e = engine(wl)
    e.step(2)
    got = e.state()
    rho = e.moments()
    e.close()
    dist, sdiff = per_subdomain(got, ref, prob)
    rr = dd.moments(ref, prob)
    m = maxnorm(rho, rr, float(np.max(np.abs(rr))))
    say(f"  subdomain distance {dist:.3e}, singular values {sdiff:.3e}, max-norm rho {m:.3e}")
    assert dist < STRICT and sdiff < STRICT and m < STRICT


def _adaptive_case(seed=23, **kw):
    args = dict(seed=seed, px=2, py=2, lnx=8, lny=8, dirs=wk.product_directions(6, 6), ranks=[3, 4, 2, 3],
                rank_mode=wk.RANK_ADAPTIVE, tol=1e-6, r_max=6, r_int_max=12, r_min=1)
    args.update(kw)
    return small_case(**args)


def test_forced_ranks_against_the_oracle_with_the_same_ranks():
    """dd_dlra_force_ranks replaces both rank rules: intermediate rank 12
    (clipped to m0 by the capacity, so the whole augmentation matrix is
    kept) and stored ranks that differ from the tolerance rule.  The oracle
    with its rank functions replaced by the same numbers (call k of a rank
    function belongs to subdomain k mod S of advection stage k div S)
    gives the same two steps to 1e-10."""
    wl = _adaptive_case()
    S_ = wl.n_sub
    t_force = [12] * (2 * S_)
    r_force = [2, 3, 3, 2] + [3, 2, 2, 3]
    calls = {"aug": 0, "trunc": 0}
    orig_aug, orig_trunc = dd.aug_rank, dd.trunc_rank

    def aug_forced(sig, r, m0, prob_):
        k = calls["aug"]
        calls["aug"] += 1
        return min(t_force[(k // S_) % 2 * S_ + k % S_], min(m0, prob_.r_int_max)), False

    def trunc_forced(sig, prob_):
        k = calls["trunc"]
        calls["trunc"] += 1
        return min(r_force[(k // S_) % 2 * S_ + k % S_], len(sig)), False

    say("case: 2x2 of 8x8, adaptive, ranks forced (t = m0, r' = 2/3 pattern), 2 steps")
    try:
        dd.aug_rank, dd.trunc_rank = aug_forced, trunc_forced
        ref, prob = oracle_steps(wl, 2)
    finally:
        dd.aug_rank, dd.trunc_rank = orig_aug, orig_trunc
    assert calls["aug"] == calls["trunc"] == 4 * S_
    e = engine(wl)
    e.force_ranks(t_force, r_force)
    e.step(2)
    got = e.state()
    r, _, _ = e.ranks()
    e.close()
    assert list(r) == r_force[S_:]
    dist, sdiff = per_subdomain(got, ref, prob)
    say(f"  ranks {list(r)}, subdomain distance {dist:.3e}, singular values {sdiff:.3e}")
    assert dist < STRICT and sdiff < STRICT


def test_rank_clamps_counted_and_latched_in_strict_mode():
    """A tolerance far below what the capacities hold (1e-14 with r_max 3,
    r_int_max 5): both rank rules clamp.  The engine counts as many clamp
    events as the oracle reports over two steps and matches its state; with
    strict_caps the first clamp latches DD_ERANK."""
    import paper_2602_14854_amd as pkg
    wl = _adaptive_case(seed=29, ranks=[3, 3, 2, 3], tol=1e-14, r_max=3, r_int_max=5)
    say("case: 2x2 of 8x8, adaptive, tol 1e-14, r_max 3, r_int_max 5, 2 steps")
    prob = dd.Problem(wl)
    st = dd.initial_state(wl)
    clamps = 0
    for _ in range(2):
        recs = {}
        st = dd.dd_step(st, prob, records=recs)
        clamps += sum(int(x["aug_clamp"]) + int(x["trunc_clamp"]) for x in recs["x"] + recs["y"])
    e = engine(wl)
    e.step(2)
    got = e.state()
    _, _, n_clamp = e.ranks()
    e.close()
    dist, _ = per_subdomain(got, st, prob)
    say(f"  clamp events: engine {n_clamp}, oracle {clamps}; subdomain distance {dist:.3e}")
    assert clamps > 0 and n_clamp == clamps
    assert dist < STRICT
    e = engine(wl, strict_caps=1)
    with pytest.raises(pkg.DDError, match="status -4"):
        e.step(1)
        e.ranks()
    e.close()
