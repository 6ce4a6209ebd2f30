"""Classic (single-domain) split projector-splitting integrator in dense-matrix
form (test infrastructure only).

One low-rank representation F = U S V^T covers the whole grid.  A step is the
Lie splitting of Section 3 with the PSI of Section 2 (K-, S-, L-step, eqs.
Kstep_general / Sstep_general / Lstep_general) applied to x-advection,
y-advection and collision in turn, explicit Euler, no augmentation and no
truncation.  The difference operators are explicit N x N matrices; the
boundary value of f is the paper's f^b (eqs. fboundary_x_L/R) with zero
inflow, i.e. the own outflow value on the outflow part.  The K-step is
upwinded in the eigenbasis of C (Appendix A), written as the split
D^- K C^+ + D^+ K C^- with C^{+/-} = P diag(max/min(lambda, 0)) P^T, and the
L-step is upwinded direction by direction (R9).

It imports nothing from the domain-decomposition oracle.
"""
from __future__ import annotations

import numpy as np


class Ops:
    def __init__(self, wl):
        assert wl.px == 1 and wl.py == 1
        self.nx, self.ny = wl.nx, wl.ny
        self.N = wl.nx * wl.ny
        self.h = (wl.x1 - wl.x0) / wl.nx
        self.w = np.asarray(wl.w, float)
        self.W = float(self.w.sum())
        self.om = (np.asarray(wl.omega_x, float), np.asarray(wl.omega_y, float))
        self.c, self.dt = float(wl.c_adv), float(wl.dt)
        self.cs = np.asarray(wl.sigma_s, float)
        self.ct = self.cs + np.asarray(wl.sigma_a, float)
        self.Q = np.asarray(wl.Q, float)
        self.Dm, self.Dp, self.Elo, self.Ehi = {}, {}, {}, {}
        for axis in (0, 1):
            self._build(axis)

    def _build(self, axis):
        nx, ny, N, h = self.nx, self.ny, self.N, self.h
        Dm = np.zeros((N, N))
        Dp = np.zeros((N, N))
        nface = ny if axis == 0 else nx
        Elo = np.zeros((N, nface))
        Ehi = np.zeros((N, nface))
        for iy in range(ny):
            for ix in range(nx):
                p = iy * nx + ix
                i_al, n_al = (ix, nx) if axis == 0 else (iy, ny)
                f = iy if axis == 0 else ix
                step = 1 if axis == 0 else nx
                Dm[p, p] += 1.0 / h
                if i_al > 0:
                    Dm[p, p - step] -= 1.0 / h
                else:
                    Elo[p, f] = 1.0
                Dp[p, p] -= 1.0 / h
                if i_al < n_al - 1:
                    Dp[p, p + step] += 1.0 / h
                else:
                    Ehi[p, f] = 1.0
        self.Dm[axis], self.Dp[axis], self.Elo[axis], self.Ehi[axis] = Dm, Dp, Elo, Ehi

    # D^-(X; g) = D^-_0 X - E_lo g / h ;  D^+(X; g) = D^+_0 X + E_hi g / h
    def dminus(self, X, g, axis):
        return self.Dm[axis] @ X - self.Elo[axis] @ g / self.h

    def dplus(self, X, g, axis):
        return self.Dp[axis] @ X + self.Ehi[axis] @ g / self.h


def _qr_u(K, o):
    Q, R = np.linalg.qr(K)
    d = np.sign(np.diag(R)); d[d == 0] = 1
    return Q * d / o.h, o.h * (d[:, None] * R)


def _qr_v(L, o):
    sw = np.sqrt(o.w)
    Q, R = np.linalg.qr(sw[:, None] * L)
    d = np.sign(np.diag(R)); d[d == 0] = 1
    return (Q * d) / sw[:, None], (d[:, None] * R).T


def advect(U, S, V, axis, o: Ops):
    w, om, c, dt, h = o.w, o.om[axis], o.c, o.dt, o.h
    C = V.T @ ((w * om)[:, None] * V)
    lam, P = np.linalg.eigh(C)
    Cp = P @ np.diag(np.maximum(lam, 0.0)) @ P.T
    Cn = P @ np.diag(np.minimum(lam, 0.0)) @ P.T
    K = U @ S
    # boundary values: zero inflow, own outflow (f^b projected on V)
    Eneg = V.T @ ((w * (om < 0))[:, None] * V)
    Epos = V.T @ ((w * (om >= 0))[:, None] * V)
    gl = o.Elo[axis].T @ K @ Eneg
    gh = o.Ehi[axis].T @ K @ Epos

    def rhs(X):
        return -c * (o.dminus(X, gl, axis) @ Cp + o.dplus(X, gh, axis) @ Cn)

    K1 = K + dt * rhs(K)
    U1, S1 = _qr_u(K1, o)
    S2 = S1 - dt * h * h * U1.T @ rhs(U1 @ S1)
    Hm = h * h * U1.T @ o.dminus(U1 @ S2, gl, axis)
    Hp = h * h * U1.T @ o.dplus(U1 @ S2, gh, axis)
    L1 = V @ S2.T - dt * c * ((np.maximum(om, 0.0)[:, None] * V) @ Hm.T
                              + (np.minimum(om, 0.0)[:, None] * V) @ Hp.T)
    V1, S3 = _qr_v(L1, o)
    return U1, S3, V1


def collide(U, S, V, o: Ops):
    w, W, dt, h = o.w, o.W, o.dt, o.h
    m = V.T @ w
    K = U @ S
    K1 = K + dt * ((o.cs / W * (K @ m))[:, None] * m[None, :] - o.ct[:, None] * K + o.Q[:, None] * m[None, :])
    U1, S1 = _qr_u(K1, o)
    Gs = h * h * U1.T @ (o.cs[:, None] * U1)
    Gt = h * h * U1.T @ (o.ct[:, None] * U1)
    q = h * h * U1.T @ o.Q
    S2 = S1 + dt * (-(Gs @ S1 @ np.outer(m, m)) / W + Gt @ S1 - np.outer(q, m))
    L = V @ S2.T
    L1 = L + dt * (np.outer(np.ones_like(w), (w @ L) @ Gs) / W - L @ Gt + np.outer(np.ones_like(w), q))
    V1, S3 = _qr_v(L1, o)
    return U1, S3, V1


def step(U, S, V, o: Ops):
    U, S, V = advect(U, S, V, 0, o)
    U, S, V = advect(U, S, V, 1, o)
    return collide(U, S, V, o)
