"""The allocation-free moments entry point (dd_dlra_moments_noalloc) against
dd_dlra_moments, through the C ABI.

Both entry points run the same arithmetic in the same order, so the scalar
flux and the current densities must agree bitwise.  The calls go in a row on
one GPU, the second on a smaller problem, so that what the first leaves in
the static scratch cannot leak into the second; the rank-64 case reaches the
largest stored rank of the scratch layout.
"""
import numpy as np
import pytest

import workloads as wk

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_14854_amd as pkg
    pkg.load_library()


def say(msg):
    print(msg, flush=True)


def case(px, py, lnx, ranks, M=(4, 4), seed=5, sig_lo=None):
    rng = np.random.default_rng(seed + 1)
    nx, ny = px * lnx, py * lnx
    n = nx * ny
    kw = {}
    if sig_lo is not None:
        def init(N, Mm, r, h, w, rng_, s):
            return wk.random_factors(N, Mm, r, h, w, rng_, sig=np.logspace(0, np.log10(sig_lo), r))
        kw = dict(rank_mode=wk.RANK_ADAPTIVE, r_fixed=max(ranks), r_max=64, r_int_max=128, r_min=1,
                  tol=1e-8, init=init)
    return wk.make_custom(nx, ny, px, py, wk.product_directions(*M), ranks, seed=seed,
                          sigma_s=rng.uniform(0, 2, n), sigma_a=rng.uniform(0, 1, n), Q=rng.uniform(0, 1, n),
                          cfl=0.5, **kw)


def noalloc_moments(e, currents):
    import torch
    n = e.nx * e.ny
    out = [torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0") for _ in range(3 if currents else 1)]
    if currents:
        e.moments_noalloc(out[0], out[1], out[2])
    else:
        e.moments_noalloc(out[0])
    e.sync()
    return [t.cpu().numpy() for t in out]


def check_against_moments(e, label):
    rho, jx, jy = e.currents()
    got = noalloc_moments(e, True)
    say(f"  {label}: rho, jx, jy bitwise {[np.array_equal(a, b) for a, b in zip(got, (rho, jx, jy))]}")
    for a, b in zip(got, (rho, jx, jy)):
        assert np.array_equal(a, b)
    (r_only,) = noalloc_moments(e, False)
    assert np.array_equal(r_only, e.moments())


def test_noalloc_moments_two_calls_in_a_row():
    from paper_2602_14854_amd import DDDLRA
    rng = np.random.default_rng(3)
    big = case(4, 4, 16, list(rng.integers(2, 9, 16)), M=(8, 8))
    small = case(2, 2, 8, [3, 1, 4, 2])
    say("case: noalloc moments, 4x4 of 16x16 (M=64, 2 steps) then 2x2 of 8x8 (M=16, 1 step)")
    with DDDLRA(big) as e1, DDDLRA(small) as e2:
        e1.step(2)
        e2.step(1)
        check_against_moments(e1, "first call, 16 subdomains")
        check_against_moments(e2, "second call, 4 subdomains")


def test_noalloc_moments_at_the_largest_rank():
    from paper_2602_14854_amd import DDDLRA
    wl = case(3, 1, 16, [62, 64, 60], M=(16, 16), sig_lo=1e-4, seed=11)
    small = case(1, 1, 8, [2], seed=7)
    say("case: noalloc moments, 3x1 of 16x16 (M=256, ranks 62/64/60) then 1x1 of 8x8")
    with DDDLRA(wl) as e1, DDDLRA(small) as e2:
        check_against_moments(e1, "ranks up to 64")
        check_against_moments(e2, "one subdomain")


def test_noalloc_rejects_more_subdomains_than_the_scratch_holds():
    from paper_2602_14854_amd import DDDLRA, DDError
    import torch
    wl = case(33, 32, 4, [1] * (33 * 32), seed=2)
    say("case: noalloc moments with 1056 subdomains (limit 1024)")
    with DDDLRA(wl) as e:
        out = torch.zeros(e.nx * e.ny, dtype=torch.float64, device="cuda:0")
        with pytest.raises(DDError, match="at most 1024 subdomains"):
            e.moments_noalloc(out)
        assert np.isfinite(e.moments()).all()
