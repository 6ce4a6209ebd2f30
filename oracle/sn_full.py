"""Full-tensor S_N reference (test infrastructure only).

The distribution is stored densely as F[iy, ix, q] on the whole grid.  One
step is the Lie splitting of Section 3 (x-advection, then y-advection, then
absorption/scattering/source), each part advanced by one explicit Euler step
(or one classic RK4 step), with the first-order upwind difference of Appendix A applied direction by
direction.  Physical boundaries are vacuum: zero inflow.  Scattering uses
c_s rho / W with rho = sum_q w_q f_q (R1, R22).

This module is written independently of the low-rank oracle (it imports
nothing from it) so that the low-rank code can be checked against it.
"""
from __future__ import annotations

import numpy as np


class Grid:
    def __init__(self, wl):
        self.nx, self.ny = wl.nx, wl.ny
        self.h = (wl.x1 - wl.x0) / wl.nx
        self.ox = np.asarray(wl.omega_x, float)
        self.oy = np.asarray(wl.omega_y, float)
        self.w = np.asarray(wl.w, float)
        self.W = float(self.w.sum())
        self.c = float(wl.c_adv)
        self.dt = float(wl.dt)
        self.ss = np.asarray(wl.sigma_s, float).reshape(wl.ny, wl.nx)
        self.st = self.ss + np.asarray(wl.sigma_a, float).reshape(wl.ny, wl.nx)
        self.Q = np.asarray(wl.Q, float).reshape(wl.ny, wl.nx)
        self.integrator = str(getattr(wl, "integrator", "euler"))


def upwind_derivative(F, axis, omega, h, inflow_lo=None, inflow_hi=None):
    """Per-direction first-order upwind derivative of F[iy, ix, q] along
    axis (0 = x, 1 = y): backward difference where omega_q > 0, forward where
    omega_q < 0, zero where omega_q = 0.  The cell beyond the grid holds
    inflow_lo / inflow_hi (arrays over the face and q) or zero."""
    ny, nx, M = F.shape
    ax = 1 if axis == 0 else 0
    D = np.zeros_like(F)
    Fm = np.moveaxis(F, ax, 0)                   # [n_along, n_across, M]
    n = Fm.shape[0]
    lo = np.zeros(Fm.shape[1:]) if inflow_lo is None else inflow_lo
    hi = np.zeros(Fm.shape[1:]) if inflow_hi is None else inflow_hi
    prev = np.concatenate([lo[None], Fm[:-1]], axis=0)
    nxt = np.concatenate([Fm[1:], hi[None]], axis=0)
    back = (Fm - prev) / h
    fwd = (nxt - Fm) / h
    Dm = np.where(omega[None, None, :] > 0, back, np.where(omega[None, None, :] < 0, fwd, 0.0))
    D = np.moveaxis(Dm, 0, ax)
    assert D.shape == (ny, nx, M) and n > 0
    return D


def advect(F, axis, g: Grid, inflow_lo=None, inflow_hi=None):
    om = g.ox if axis == 0 else g.oy
    return F - g.dt * g.c * om[None, None, :] * upwind_derivative(F, axis, om, g.h, inflow_lo, inflow_hi)


def advect_operator(F, axis, g: Grid, inflow_lo=None, inflow_hi=None):
    """A(F) = -c omega D F (affine through the inflow values)."""
    om = g.ox if axis == 0 else g.oy
    return -g.c * om[None, None, :] * upwind_derivative(F, axis, om, g.h, inflow_lo, inflow_hi)


def collide_operator(F, g: Grid, with_source=True):
    rho = F @ g.w
    out = (g.ss / g.W * rho)[:, :, None] - g.st[:, :, None] * F
    if with_source:
        out = out + g.Q[:, :, None]
    return out


def collide(F, g: Grid):
    return F + g.dt * collide_operator(F, g)


def _rk4(f, y, dt):
    # classic four-stage Runge-Kutta step for y' = f(y)
    a = f(y)
    b = f(y + (dt / 2) * a)
    c = f(y + (dt / 2) * b)
    e = f(y + dt * c)
    return y + (dt / 6) * (a + 2 * b + 2 * c + e)


def step(F, g: Grid):
    """One Lie-split S_N step: x, then y, then collision, each part advanced
    by one explicit Euler step or one classic RK4 step (g.integrator)."""
    if g.integrator == "rk4":
        F = _rk4(lambda X: advect_operator(X, 0, g), F, g.dt)
        F = _rk4(lambda X: advect_operator(X, 1, g), F, g.dt)
        return _rk4(lambda X: collide_operator(X, g), F, g.dt)
    F = advect(F, 0, g)
    F = advect(F, 1, g)
    return collide(F, g)


def from_flat(Fflat, wl):
    return Fflat.reshape(wl.ny, wl.nx, -1)


def to_flat(F):
    return F.reshape(-1, F.shape[2])
