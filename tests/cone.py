"""Oracle steps restricted to the domain of dependence of a few subdomains.

Within a stage a subdomain reads only its two neighbours along the stage's
axis (as they were at the start of the stage), so the factors of a window of
subdomains after n steps depend only on a neighbourhood n subdomains wide
around it.  cone_steps advances just that neighbourhood with the oracle's
own stage functions, which makes oracle parity affordable at the full size
of the largest grids.
"""
from oracle import ddlra as dd


def _closed(prob, valid, axis):
    """Subdomains of `valid` whose neighbours along axis are valid or absent."""
    out = set()
    for s in valid:
        ok = True
        for side in (-1, 1):
            n = prob.neighbour(s, axis, side)
            if n is not None and n not in valid:
                ok = False
        if ok:
            out.add(s)
    return out


def window(prob, sx0, sx1, sy0, sy1):
    """Subdomains with sx0 <= sx <= sx1 and sy0 <= sy <= sy1."""
    return {sy * prob.px + sx for sy in range(sy0, sy1 + 1) for sx in range(sx0, sx1 + 1)}


def cone_steps(state, prob, target, nsteps):
    """Advance the oracle nsteps steps on the domain of dependence of the
    subdomains in target.  Returns (state, valid): the factors of every
    subdomain in valid (a superset of target) are those of the full oracle
    run; the others are stale."""
    valid = set(target)
    for _ in range(nsteps):  # grow the start set by one subdomain per step along x, then y
        for axis in (0, 1):
            grown = set(valid)
            for s in valid:
                for side in (-1, 1):
                    n = prob.neighbour(s, axis, side)
                    if n is not None:
                        grown.add(n)
            valid = grown
    for _ in range(nsteps):
        vx = _closed(prob, valid, 0)
        state = dd.stage_advect(state, 0, prob, only=vx)
        vy = _closed(prob, vx, 1)
        state = dd.stage_advect(state, 1, prob, only=vy)
        state = dd.stage_collision(state, prob, only=vy)
        valid = vy
    assert set(target) <= valid
    return state, valid
