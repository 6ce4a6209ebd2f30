"""One DD-DLRA time step in plain FP64 NumPy (test infrastructure only).

Follows the paper: Section 3 (domain decomposition low-rank algorithm),
Algorithms 1-6, the inflow boundary projection (eq. generate_Kboundary and
its y counterpart), and Appendix A (upwinding of the K-step through the
eigen-decomposition of C).  Readings used where the paper is silent:

  R1/R22  general direction set (omega_x, omega_y, w); scattering c_s rho / W
          with W = sum(w) (the 2x1-D model has W = 2 pi).
  R3      positive class of the inflow indicator is omega >= 0.
  R4      weighted inner products: h^2 U^T U = I and V^T diag(w) V = I.
  R5      the ghost value of a face is the neighbour's adjacent cell column
          (inflow part) and the subdomain's own face column (outflow part).
  R6      within a stage every subdomain sees its neighbours' factors as they
          were at the start of the stage; stages are bulk-synchronous.
  R7      the boundary data K^b are computed once per stage and frozen.
  R8      x uses omega_x, y uses omega_y; eigenvalue 0 contributes nothing.
  R9      the S-step is the Galerkin projection of the K-step operator; the
          L-step upwinds each direction by the sign of its own omega.
  R10     explicit Euler for every K, S and L substep; the classic
          four-stage Runge-Kutta method (Section 4 states that the paper's
          runs use it) is available per problem, each substep integrated
          over dt with its boundary data frozen; so is the exact flow of
          each substep (matrix exponential of its affine right-hand side,
          tiny grids only), the sub-flows under which the projector-splitting
          integrator is exact (Section 2).
  R12     Algorithm 4's top block of S-hat is S^0 V^{0T} W V-hat.
  R14/R15 rank rules (see aug_rank / trunc_rank).
  R16     the collision stage does not truncate.
  R17     a physical vacuum face has zero inflow; the own outflow part stays.
  R33     a physical inflow face (the prescribed inflow of Section 4's
          Hohlraum and boundary point-source problems, f_in = A B^T along the
          face) acts as a neighbour: a layer one cell thick outside the face
          holding f_in, with the factors U_v = Q_a / h (on its cells next to
          the face), S_v = h R_a, V_v = B from the thin QR A_s = Q_a R_a of the
          subdomain's part of A.  It supplies the inflow part of the ghost
          values, and V_v S_v^T = h B R_a^T joins L0 in the augmentation, as a
          neighbour's V_n S_n^T does.
"""
from __future__ import annotations

import numpy as np

RANK_FIXED = 0
RANK_ADAPTIVE = 1


# ----------------------------------------------------------------------------
# problem geometry
# ----------------------------------------------------------------------------

class Problem:
    """Grid, subdomain layout, directions and coefficients of one run.

    Built from any object with the workload attributes (nx, ny, px, py, x0, x1,
    omega_x, omega_y, w, c_adv, sigma_s, sigma_a, Q, dt and rank settings)."""

    def __init__(self, wl):
        self.nx, self.ny, self.px, self.py = wl.nx, wl.ny, wl.px, wl.py
        self.lnx, self.lny = wl.nx // wl.px, wl.ny // wl.py
        self.N = self.lnx * self.lny
        self.h = (wl.x1 - wl.x0) / wl.nx
        self.omega = (np.asarray(wl.omega_x, float), np.asarray(wl.omega_y, float))
        self.w = np.asarray(wl.w, float)
        self.M = self.w.shape[0]
        self.W = float(np.sum(self.w))
        self.c = float(wl.c_adv)
        self.dt = float(wl.dt)
        self.inflow = list(getattr(wl, "inflow", None) or [None] * 4)
        self.rank_mode = int(wl.rank_mode)
        self.r_fixed = int(wl.r_fixed)
        self.r_min, self.r_max = int(wl.r_min), int(wl.r_max)
        self.r_int_max = int(wl.r_int_max)
        self.tol = float(wl.tol)
        self.tol_aug_rel = float(wl.tol_aug_rel)
        self.integrator = str(getattr(wl, "integrator", "euler"))
        if self.integrator not in ("euler", "rk4", "expm"):
            raise ValueError("integrator must be 'euler', 'rk4' or 'expm'")
        n_sub = wl.px * wl.py
        self.sigma_s, self.sigma_t, self.Q = [], [], []
        for s in range(n_sub):
            cells = self.local_cells(s)
            ss = np.asarray(wl.sigma_s, float)[cells]
            sa = np.asarray(wl.sigma_a, float)[cells]
            self.sigma_s.append(ss)
            self.sigma_t.append(ss + sa)          # c_t = c_a + c_s (Section 2)
            self.Q.append(np.asarray(wl.Q, float)[cells])

    @property
    def n_sub(self):
        return self.px * self.py

    def local_cells(self, s):
        sx, sy = s % self.px, s // self.px
        iy = sy * self.lny + np.arange(self.lny)
        ix = sx * self.lnx + np.arange(self.lnx)
        return (iy[:, None] * self.nx + ix[None, :]).ravel()

    def neighbour(self, s, axis, side):
        """Subdomain next to s along axis (0 = x, 1 = y) on side -1 (left /
        bottom) or +1 (right / top); None at the physical boundary."""
        sx, sy = s % self.px, s // self.px
        if axis == 0:
            sx += side
            if sx < 0 or sx >= self.px:
                return None
        else:
            sy += side
            if sy < 0 or sy >= self.py:
                return None
        return sy * self.px + sx

    def virtual_neighbour(self, s, axis, side):
        """(U_v, S_v, V_v) of the inflow layer outside a physical inflow face
        of subdomain s (R33), or None (an interior face or a vacuum face).
        U_v is nonzero only on its face next to s."""
        sx, sy = s % self.px, s // self.px
        if axis == 0:
            if (side < 0 and sx > 0) or (side > 0 and sx < self.px - 1):
                return None
            f = 0 if side < 0 else 1
            pos = sy * self.lny + np.arange(self.lny)
        else:
            if (side < 0 and sy > 0) or (side > 0 and sy < self.py - 1):
                return None
            f = 2 if side < 0 else 3
            pos = sx * self.lnx + np.arange(self.lnx)
        if self.inflow[f] is None:
            return None
        A, B = self.inflow[f]
        As = np.asarray(A, float)[pos]
        Qa, Ra = np.linalg.qr(As)
        U = np.zeros((self.N, As.shape[1]))
        U[self.face(axis, side < 0)] = Qa / self.h   # its cells next to s
        return U, self.h * Ra, np.asarray(B, float)

    def face(self, axis, high):
        """Local cell indices of a subdomain face, ordered along the face:
        axis 0 -> the column ix = 0 (high=False) or ix = lnx-1, ordered by iy;
        axis 1 -> the row iy = 0 or iy = lny-1, ordered by ix."""
        if axis == 0:
            ix = self.lnx - 1 if high else 0
            return np.arange(self.lny) * self.lnx + ix
        iy = self.lny - 1 if high else 0
        return iy * self.lnx + np.arange(self.lnx)


# ----------------------------------------------------------------------------
# first-order upwind differences on a subdomain grid (Appendix A)
# ----------------------------------------------------------------------------

def backward_diff(X, axis, ghost, prob):
    """(D^- X)[cell] = (X[cell] - X[cell - e_axis]) / h, with the ghost row
    standing in for the cell before the first one.  X: N x k, ghost: face x k."""
    k = X.shape[1]
    G = X.reshape(prob.lny, prob.lnx, k)
    if axis == 0:
        prev = np.concatenate([ghost.reshape(prob.lny, 1, k), G[:, :-1, :]], axis=1)
    else:
        prev = np.concatenate([ghost.reshape(1, prob.lnx, k), G[:-1, :, :]], axis=0)
    return ((G - prev) / prob.h).reshape(prob.N, k)


def forward_diff(X, axis, ghost, prob):
    """(D^+ X)[cell] = (X[cell + e_axis] - X[cell]) / h, with the ghost row
    standing in for the cell after the last one."""
    k = X.shape[1]
    G = X.reshape(prob.lny, prob.lnx, k)
    if axis == 0:
        nxt = np.concatenate([G[:, 1:, :], ghost.reshape(prob.lny, 1, k)], axis=1)
    else:
        nxt = np.concatenate([G[1:, :, :], ghost.reshape(1, prob.lnx, k)], axis=0)
    return ((nxt - G) / prob.h).reshape(prob.N, k)


def kstep_rhs(K, P, lam, Kb_lo, Kb_hi, axis, prob):
    """Right-hand side of the advection K-step, d/dt K = -c_adv D_X K C, with
    C = P diag(lam) P^T (Appendix A): the columns of K P whose eigenvalue is
    positive take the backward difference, negative ones the forward
    difference, and the result is multiplied back by diag(lam) P^T (R8)."""
    Kt = K @ P
    gl = Kb_lo @ P
    gh = Kb_hi @ P
    D = np.zeros_like(Kt)
    for m in range(Kt.shape[1]):
        if lam[m] > 0:
            D[:, m:m + 1] = backward_diff(Kt[:, m:m + 1], axis, gl[:, m:m + 1], prob)
        elif lam[m] < 0:
            D[:, m:m + 1] = forward_diff(Kt[:, m:m + 1], axis, gh[:, m:m + 1], prob)
    return -prob.c * (D * lam[None, :]) @ P.T


def direction_rhs(F, omega, G_lo, G_hi, axis, prob):
    """Full-tensor upwind advection -c_adv omega_q D F[:, q] for every
    direction q, each upwinded by the sign of its own omega_q (R9); G_lo and
    G_hi are the ghost rows (face x M)."""
    D = np.zeros_like(F)
    for q in range(F.shape[1]):
        if omega[q] > 0:
            D[:, q:q + 1] = backward_diff(F[:, q:q + 1], axis, G_lo[:, q:q + 1], prob)
        elif omega[q] < 0:
            D[:, q:q + 1] = forward_diff(F[:, q:q + 1], axis, G_hi[:, q:q + 1], prob)
    return -prob.c * D * omega[None, :]


# ----------------------------------------------------------------------------
# orthonormalisation (QR with non-negative diagonal, R4/R18)
# ----------------------------------------------------------------------------

def _sign_fix(Q, R):
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :], d[:, None] * R


def qr_spatial(K, prob):
    """K = U S with h^2 U^T U = I (Householder QR of K: U = Q / h, S = h R)."""
    Q, R = np.linalg.qr(K)
    Q, R = _sign_fix(Q, R)
    return Q / prob.h, prob.h * R


def qr_angular(L, prob):
    """L = V S^T with V^T diag(w) V = I (QR of diag(sqrt w) L: V = Q / sqrt w,
    S = R^T).  Used for the final step of Algorithms 1-3."""
    sw = np.sqrt(prob.w)
    Q, R = np.linalg.qr(sw[:, None] * L)
    Q, R = _sign_fix(Q, R)
    return Q / sw[:, None], R.T


# ----------------------------------------------------------------------------
# rank rules
# ----------------------------------------------------------------------------

def tail_rank(sig, tol):
    """Smallest k with (sum_{j > k} sig_j^2)^(1/2) <= tol (Algorithms 4 and 5)."""
    n = len(sig)
    for k in range(n + 1):
        if np.sqrt(np.sum(np.asarray(sig[k:]) ** 2)) <= tol:
            return k
    return n


def aug_rank(sig, r, m0, prob):
    """Intermediate rank after augmentation (Algorithm 4, step 3, and R14):
    t = max(r, tail rank) clamped to min(m0, r_int_max).  Fixed-rank mode uses
    the relative tolerance tol_aug_rel * sigma_1, adaptive mode uses tol.
    Returns (t, clamped)."""
    if prob.rank_mode == RANK_FIXED:
        tol = prob.tol_aug_rel * (sig[0] if len(sig) else 0.0)
    else:
        tol = prob.tol
    t = max(r, tail_rank(sig, tol))
    cap = min(m0, prob.r_int_max)
    return min(t, cap), t > cap


def trunc_rank(sig, prob):
    """Stored rank after truncation (Algorithm 5, step 2, and R15): fixed mode
    keeps r_fixed; adaptive mode takes the tail rank, at least r_min and at
    most r_max.  Returns (r', clamped)."""
    t = len(sig)
    if prob.rank_mode == RANK_FIXED:
        return min(prob.r_fixed, t), False
    k = max(prob.r_min, tail_rank(sig, prob.tol))
    cap = min(prob.r_max, t)
    return min(k, cap), k > cap


# ----------------------------------------------------------------------------
# Algorithm 4: augmentation
# ----------------------------------------------------------------------------

def augment(U, S, V, nbrs, prob, U_rand=None):
    """Algorithm 4 for one subdomain.

    nbrs: list of (V_n, S_n) of the (at most two) neighbours along the stage's
    axis, taken at the start of the stage (R6, R13: the neighbour's full S).
    Returns (K, V_hat, t, sig, clamped) where K = U^1 S^1 is the K-step's
    initial value in the basis V_hat.

    With U_rand (N x >= t-r random columns, an input) the steps are done
    literally: U-hat = [U, U_rand], S-hat = [S V^T W V-hat; 0], QR of both
    bases, S^1 = S_U S-hat S_V^T.  Without it, K = U S (V^T W V-hat), which is
    the same product because the random columns meet a zero block (R12)."""
    w = prob.w
    sw = np.sqrt(w)
    L0 = np.hstack([V @ S.T] + [Vn @ Sn.T for (Vn, Sn) in nbrs])       # step 1
    Vw, sig, _ = np.linalg.svd(sw[:, None] * L0, full_matrices=False)  # step 2 (R4)
    r = U.shape[1]
    t, clamped = aug_rank(sig, r, L0.shape[1], prob)                   # step 3
    V_hat = Vw[:, :t] / sw[:, None]                                     # step 4
    top = S @ (V.T @ (w[:, None] * V_hat))                             # S V^T W V-hat
    if U_rand is None:
        K = U @ top
    else:
        U_hat = np.hstack([U, U_rand[:, : t - r]])                      # step 5
        S_hat = np.vstack([top, np.zeros((t - r, t))])
        U1, S_U = qr_spatial(U_hat, prob)                               # step 6: U-hat = U^1 S_U
        Q_V, R_V = np.linalg.qr(sw[:, None] * V_hat)                    # V-hat = V^1 S_V
        Q_V, R_V = _sign_fix(Q_V, R_V)
        V_hat = Q_V / sw[:, None]
        S1 = S_U @ S_hat @ R_V.T
        K = U1 @ S1
    return K, V_hat, t, sig, clamped


# ----------------------------------------------------------------------------
# inflow boundary data (eq. generate_Kboundary and its y counterpart)
# ----------------------------------------------------------------------------

def neighbour_factors(s, axis, side, snapshot, prob):
    """Factors of the subdomain next to s on that side as they were at the
    start of the stage (R6), the inflow layer of a physical inflow face
    (R33), or None (vacuum)."""
    n = prob.neighbour(s, axis, side)
    if n is not None:
        return snapshot[n]
    return prob.virtual_neighbour(s, axis, side)


def boundary_K(s, axis, K, V_hat, snapshot, prob):
    """K^b on the low and high faces of subdomain s for one advection stage.

    Low face: inflow for omega >= 0 comes from the low neighbour's K at its
    high face, projected with <1_{omega>=0} V^n_l, V-hat_j>; the outflow part
    (omega < 0) is this subdomain's own K at its low face projected with
    <1_{omega<0} V-hat_l, V-hat_j>.  The high face mirrors it.  A physical
    vacuum face contributes no inflow (R17); a physical inflow face
    contributes its prescribed inflow through its layer's factors (R33)."""
    w = prob.w
    om = prob.omega[axis]
    pos = (om >= 0).astype(float)           # R3
    neg = 1.0 - pos
    lo_face = prob.face(axis, False)
    hi_face = prob.face(axis, True)
    Kb_lo = K[lo_face] @ (V_hat.T @ ((w * neg)[:, None] * V_hat))
    Kb_hi = K[hi_face] @ (V_hat.T @ ((w * pos)[:, None] * V_hat))
    f_lo = neighbour_factors(s, axis, -1, snapshot, prob)
    f_hi = neighbour_factors(s, axis, +1, snapshot, prob)
    if f_lo is not None:
        Un, Sn, Vn = f_lo
        Kb_lo = Kb_lo + (Un[hi_face] @ Sn) @ (Vn.T @ ((w * pos)[:, None] * V_hat))
    if f_hi is not None:
        Un, Sn, Vn = f_hi
        Kb_hi = Kb_hi + (Un[lo_face] @ Sn) @ (Vn.T @ ((w * neg)[:, None] * V_hat))
    return Kb_lo, Kb_hi


# ----------------------------------------------------------------------------
# time integration of one substep
# ----------------------------------------------------------------------------

def rk4(f, y0, dt):
    """One step of the classic four-stage Runge-Kutta method for y' = f(y)
    (the substeps are autonomous: their boundary data are frozen, R7)."""
    k1 = f(y0)
    k2 = f(y0 + 0.5 * dt * k1)
    k3 = f(y0 + 0.5 * dt * k2)
    k4 = f(y0 + dt * k3)
    return y0 + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def exact_flow(f, y0, dt):
    """Exact solution at time dt of the affine ODE y' = f(y) = A y + b
    (every substep of Algorithms 1-3 is affine in its unknown once the
    boundary data are frozen).  A and b are read off f (b = f(0), column k
    of A = f(e_k) - b) and the flow is exp(dt Z) [y0; 1] with
    Z = [[A, b], [0, 0]].  Dense in y0.size: for tiny grids only."""
    import scipy.linalg
    shp = y0.shape
    n = y0.size
    b = np.asarray(f(np.zeros(shp))).ravel()
    Z = np.zeros((n + 1, n + 1))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        Z[:n, k] = np.asarray(f(e.reshape(shp))).ravel() - b
    Z[:n, n] = b
    y = scipy.linalg.expm(dt * Z) @ np.append(y0.ravel(), 1.0)
    return y[:n].reshape(shp)


def integrate(f, y0, prob):
    """One substep of length dt with the problem's integrator (R10)."""
    if prob.integrator == "rk4":
        return rk4(f, y0, prob.dt)
    if prob.integrator == "expm":
        return exact_flow(f, y0, prob.dt)
    return y0 + prob.dt * f(y0)


# ----------------------------------------------------------------------------
# Algorithms 1 and 2: projector splitting for x / y advection
# ----------------------------------------------------------------------------

def psi_advect(K0, V_hat, Kb_lo, Kb_hi, axis, prob, rec=None):
    """Algorithm 1 (axis 0) or Algorithm 2 (axis 1) with explicit Euler, RK4
    or exact substeps (R10).

    Returns (U^1, S^3, V^1) with F = U^1 S^3 V^{1T}."""
    w = prob.w
    om = prob.omega[axis]
    dt, h = prob.dt, prob.h
    C = V_hat.T @ ((w * om)[:, None] * V_hat)        # <V_j, v V_k> (Appendix A, R8)
    lam, P = np.linalg.eigh(C)
    rk = prob.integrator != "euler"   # RK4 or exact sub-flows
    # step 1: K-step (eq. advx_evolK) with frozen boundary values
    if rk:
        K1 = integrate(lambda K: kstep_rhs(K, P, lam, Kb_lo, Kb_hi, axis, prob), K0, prob)
    else:
        K1 = K0 + dt * kstep_rhs(K0, P, lam, Kb_lo, Kb_hi, axis, prob)
    # step 2: QR
    U1, S1 = qr_spatial(K1, prob)
    # step 3: S-step (eq. advx_evolS), integrated with the opposite sign
    if rk:
        S2 = integrate(lambda S: -(h * h) * (U1.T @ kstep_rhs(U1 @ S, P, lam, Kb_lo, Kb_hi, axis, prob)),
                       S1, prob)
    else:
        S2 = S1 - dt * (h * h) * (U1.T @ kstep_rhs(U1 @ S1, P, lam, Kb_lo, Kb_hi, axis, prob))
    # step 4: L-step (eq. advx_evolL) from L = V-hat S^{2T}; the per-direction
    # boundary value of f is K^b V-hat^T (R9)
    G_lo, G_hi = Kb_lo @ V_hat.T, Kb_hi @ V_hat.T
    if rk:
        L1 = integrate(lambda L: ((h * h) * (U1.T @ direction_rhs(U1 @ L.T, om, G_lo, G_hi, axis, prob))).T,
                       V_hat @ S2.T, prob)
    else:
        F2 = U1 @ S2 @ V_hat.T
        A = direction_rhs(F2, om, G_lo, G_hi, axis, prob)
        L1 = V_hat @ S2.T + dt * ((h * h) * (U1.T @ A)).T
    # step 5: QR
    V1, S3 = qr_angular(L1, prob)
    if rec is not None:
        rec.update(C=C, lam=lam, P=P, K1=K1, U1=U1, S1=S1, S2=S2, L1=L1, V1=V1, S3=S3)
    return U1, S3, V1


# ----------------------------------------------------------------------------
# Algorithm 5: truncation
# ----------------------------------------------------------------------------

def truncate(U, S, V, prob):
    """Algorithm 5: SVD of S, rank rule, rotate and cut both bases."""
    Ut, sig, Vtt = np.linalg.svd(S)
    rp, clamped = trunc_rank(sig, prob)
    return U @ Ut[:, :rp], np.diag(sig[:rp]), V @ Vtt.T[:, :rp], sig, clamped


# ----------------------------------------------------------------------------
# Algorithm 3: absorption, scattering and source
# ----------------------------------------------------------------------------

def psi_collision(U, S, V, s, prob, rec=None):
    """Algorithm 3 with explicit Euler, RK4 or exact substeps (R10), eqs.
    coll_evolK/S/L; 1/(2 pi) becomes 1/W (R1, R22)."""
    w, W, dt, h = prob.w, prob.W, prob.dt, prob.h
    cs, ct, Qs = prob.sigma_s[s], prob.sigma_t[s], prob.Q[s]
    m = V.T @ w                                         # <V_j>
    K = U @ S
    rk = prob.integrator != "euler"   # RK4 or exact sub-flows
    # step 1: K-step
    def fK(K):
        return (cs / W)[:, None] * (K @ m)[:, None] * m[None, :] - ct[:, None] * K + Qs[:, None] * m[None, :]
    K1 = integrate(fK, K, prob) if rk else K + dt * fK(K)
    # step 2: QR
    U1, S1 = qr_spatial(K1, prob)
    # step 3: S-step
    Gs = (h * h) * (U1.T @ (cs[:, None] * U1))          # <U_i, c_s U_l>
    Gt = (h * h) * (U1.T @ (ct[:, None] * U1))          # <U_i, c_t U_l>
    q = (h * h) * (U1.T @ Qs)                           # <U_i, Q>
    def fS(S):
        return -(1.0 / W) * Gs @ S @ np.outer(m, m) + Gt @ S - np.outer(q, m)
    S2 = integrate(fS, S1, prob) if rk else S1 + dt * fS(S1)
    # step 4: L-step from L = V S^{2T}
    L = V @ S2.T
    ones = np.ones(prob.M)
    def fL(L):
        return (1.0 / W) * np.outer(ones, (w @ L) @ Gs.T) - L @ Gt.T + np.outer(ones, q)
    L1 = integrate(fL, L, prob) if rk else L + dt * fL(L)
    # step 5: QR
    V1, S3 = qr_angular(L1, prob)
    if rec is not None:
        rec.update(m=m, K1=K1, U1=U1, S1=S1, S2=S2, L1=L1, V1=V1, S3=S3, Gs=Gs, Gt=Gt, q=q)
    return U1, S3, V1


# ----------------------------------------------------------------------------
# stages and the full step (Algorithm 6)
# ----------------------------------------------------------------------------

def stage_advect(state, axis, prob, rng=None, records=None, only=None):
    """Augment, advect and truncate every subdomain for one direction
    (Algorithm 6, steps 1-3 for x, 4-6 for y), all from a snapshot of the
    factors at the start of the stage (R6).  rng, if given, draws U_rand for
    the literal form of Algorithm 4.  only, if given, is a set of
    subdomains: the others keep their input factors (to follow a few
    subdomains of a large grid through their domain of dependence)."""
    snapshot = [tuple(f) for f in state]
    new = []
    for s in range(prob.n_sub):
        U, S, V = snapshot[s]
        if only is not None and s not in only:
            new.append((U, S, V))
            if records is not None:
                records.append(None)
            continue
        nbrs = []
        for side in (-1, +1):
            fn = neighbour_factors(s, axis, side, snapshot, prob)
            if fn is not None:
                nbrs.append((fn[2], fn[1]))
        U_rand = None
        if rng is not None:
            U_rand = rng.standard_normal((prob.N, prob.r_int_max + 1))
        K0, V_hat, t, sig_aug, aug_clamp = augment(U, S, V, nbrs, prob, U_rand)
        Kb_lo, Kb_hi = boundary_K(s, axis, K0, V_hat, snapshot, prob)
        rec = {} if records is not None else None
        U1, S3, V1 = psi_advect(K0, V_hat, Kb_lo, Kb_hi, axis, prob, rec)
        Un, Sn, Vn, sig_tr, tr_clamp = truncate(U1, S3, V1, prob)
        if records is not None:
            rec.update(t=t, sig_aug=sig_aug, V_hat=V_hat, K0=K0, Kb_lo=Kb_lo, Kb_hi=Kb_hi,
                       sig_trunc=sig_tr, r_new=Sn.shape[0], aug_clamp=aug_clamp,
                       trunc_clamp=tr_clamp)
            records.append(rec)
        new.append((Un, Sn, Vn))
    return new


def stage_collision(state, prob, records=None, only=None):
    """Algorithm 6, step 7: Algorithm 3 on every subdomain, no truncation
    (R16); only as in stage_advect."""
    new = []
    for s in range(prob.n_sub):
        U, S, V = state[s]
        if only is not None and s not in only:
            new.append((U, S, V))
            if records is not None:
                records.append(None)
            continue
        rec = {} if records is not None else None
        new.append(psi_collision(U, S, V, s, prob, rec))
        if records is not None:
            records.append(rec)
    return new


def dd_step(state, prob, rng=None, records=None):
    """One time step of Algorithm 6 on all subdomains.

    state: list of (U, S, V) per subdomain.  records, if a dict, receives the
    per-stage, per-subdomain intermediates under keys 'x', 'y', 'c'."""
    rx = [] if records is not None else None
    ry = [] if records is not None else None
    rc = [] if records is not None else None
    state = stage_advect(state, 0, prob, rng, rx)
    state = stage_advect(state, 1, prob, rng, ry)
    state = stage_collision(state, prob, rc)
    if records is not None:
        records.update(x=rx, y=ry, c=rc)
    return state


def initial_state(wl):
    return [(np.array(u, float), np.array(s, float), np.array(v, float))
            for u, s, v in zip(wl.U0, wl.S0, wl.V0)]


def run(wl, n_steps, rng=None):
    prob = Problem(wl)
    state = initial_state(wl)
    for _ in range(n_steps):
        state = dd_step(state, prob, rng)
    return state


# ----------------------------------------------------------------------------
# observables
# ----------------------------------------------------------------------------

def moments(state, prob):
    """Scalar flux rho = int f dOmega = sum_q w_q f_q (Section 2), assembled
    on the global grid [ny*nx]."""
    rho = np.zeros(prob.nx * prob.ny)
    for s, (U, S, V) in enumerate(state):
        rho[prob.local_cells(s)] = U @ (S @ (V.T @ prob.w))
    return rho


def currents(state, prob):
    """First angular moments, the current density j = int Omega f dOmega:
    jx = sum_q w_q Omega_x,q f_q and jy likewise, assembled on the global
    grid [ny*nx] (the flux of the transported quantity through a face)."""
    jx = np.zeros(prob.nx * prob.ny)
    jy = np.zeros(prob.nx * prob.ny)
    for s, (U, S, V) in enumerate(state):
        cells = prob.local_cells(s)
        jx[cells] = U @ (S @ (V.T @ (prob.w * prob.omega[0])))
        jy[cells] = U @ (S @ (V.T @ (prob.w * prob.omega[1])))
    return jx, jy


def assemble(state, prob):
    """The full distribution F (global cells x directions); for tiny grids."""
    F = np.zeros((prob.nx * prob.ny, prob.M))
    for s, (U, S, V) in enumerate(state):
        F[prob.local_cells(s)] = U @ S @ V.T
    return F


def factored_dist2(a, b, prob):
    """||F_a - F_b||^2 in the weighted L2 norm (the paper's error norm up to
    the constant ||1||), from the factors only.  F_a - F_b =
    [U_a U_b] diag(S_a, -S_b) [V_a V_b]^T; QR of the two stacked (weighted)
    bases reduces it to a small matrix, which avoids the cancellation floor
    of ||a||^2 + ||b||^2 - 2<a, b>."""
    Ua, Sa, Va = a
    Ub, Sb, Vb = b
    sw = np.sqrt(prob.w)
    _, Ru = np.linalg.qr(prob.h * np.hstack([Ua, Ub]))
    _, Rv = np.linalg.qr(sw[:, None] * np.hstack([Va, Vb]))
    ra, rb = Sa.shape[0], Sb.shape[0]
    D = np.zeros((ra + rb, ra + rb))
    D[:ra, :ra] = Sa
    D[ra:, ra:] = -Sb
    return float(np.sum((Ru @ D @ Rv.T) ** 2))


def state_rel_error(a, b, prob):
    """sqrt(sum_k ||F_a,k - F_b,k||^2) / sqrt(sum_k ||F_b,k||^2)."""
    num = sum(max(factored_dist2(x, y, prob), 0.0) for x, y in zip(a, b))
    den = sum(float(np.sum(y[1] ** 2)) for y in b)
    return float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num))
