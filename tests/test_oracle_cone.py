"""The domain-of-dependence driver (tests/cone.py) reproduces the full
oracle run on its target subdomains exactly: it only skips work whose
results the target never reads."""
import numpy as np

import workloads as wk
from oracle import ddlra as dd
from cone import cone_steps, window


def test_cone_matches_full_run():
    wl = wk.make_custom(28, 28, 7, 7, wk.product_directions(4, 4), [3] * 49, seed=21,
                        sigma_s=np.full(784, 0.7), sigma_a=np.full(784, 0.2), Q=np.zeros(784))
    prob = dd.Problem(wl)
    full = dd.initial_state(wl)
    for _ in range(2):
        full = dd.dd_step(full, prob)
    target = window(prob, 3, 3, 2, 3)
    got, valid = cone_steps(dd.initial_state(wl), prob, target, 2)
    assert len(valid) < prob.n_sub
    for s in target:
        for a, b in zip(got[s], full[s]):
            assert np.array_equal(a, b)
