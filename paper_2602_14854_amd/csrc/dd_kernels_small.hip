// Small dense FP64 kernels of the DD-DLRA step: one workgroup per subdomain
// works on matrices of at most 64 x 64 (the intermediate rank t or the
// augmentation width m0).  They add the tall-skinny kernels' partial sums in
// a fixed order, run the serial linear algebra (two-sided Jacobi
// eigensolver, Cholesky, triangular inverse) and form the coefficient
// matrices of the next tall-skinny pass.
#include "dd_dense.h"

namespace dd {

constexpr int CAPR = 21;

// ---------------------------------------------------------------- augmentation

// SVD of the weighted augmentation matrix A = sqrt(w) L0 (Algorithm 4, steps
// 2-4) from its Cholesky-QR factor A = Q Racc (Racc = R P^T, pivoted in the
// first pass): the one-sided Jacobi on X = Racc^T, X W = B with orthogonal
// columns, gives Racc = W Sigma Btilde^T, so the right singular vectors of A
// are the normalised columns of B and the singular values their norms (the
// pivoting makes the sweeps converge fast; the rotations themselves are not
// needed).  Then the rank rule of step 3 and the coefficients of
// sqrt(w) V-hat = A B[:, :t] Sigma^-2.
__global__ __launch_bounds__(NTHR) void s_aug_svd(Dev d, int axis, int sd0) {
  const int s = sd0 + blockIdx.x;
  const int m0 = m0_of(d, s, axis);
  const int r = d.rank[s];
  __shared__ double B[LDA * CAP];
  __shared__ double sig[CAP];
  __shared__ double nrm[CAP];
  __shared__ int perm[CAP];
  __shared__ int tsh;
  double* sm = small_of(d, s);
  {
    // B = Racc^T, eight loads in flight per thread
    const double* Ra = sm + d.oRaccA;
    const int n = m0 * m0;
    for (int base = threadIdx.x; base < n; base += 8 * NTHR) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int idx = base + u * NTHR;
        v[u] = idx < n ? Ra[(idx % m0) + (idx / m0) * d.MA] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int idx = base + u * NTHR;
        if (idx < n) B[(idx / m0) + (idx % m0) * LDA] = v[u];
      }
    }
    __syncthreads();
  }
  jacobi_1s(d, B, m0, m0, nullptr, 1e-14, 1e-15, 40);
  col_norms(B, m0, m0, nrm);
  sort_desc(nrm, m0, perm);
  for (int j = threadIdx.x; j < m0; j += NTHR) sig[j] = nrm[perm[j]];
  __syncthreads();
  if (threadIdx.x == 0) {
    int t;
    const int cap = min(min(m0, d.r_int_max), d.T);
    if (d.forced && d.force[axis * d.nsub + s] > 0) {
      t = min(d.force[axis * d.nsub + s], cap);
    } else {
      const double tol = (d.rank_mode == 0) ? d.tol_aug_rel * sig[0] : d.tol;
      t = max(r, tail_rank(sig, m0, tol));
      if (t > cap) {
        t = cap;
        atomicAdd(d.clamps, 1ull);
        if (d.strict) atomicOr(d.flags, FLAG_RANK_CLAMP);
      }
    }
    if (t < 1) t = 1;
    tsh = t;
    d.tdim[s] = t;
    if (t > d.tmax[s]) d.tmax[s] = t;
  }
  __syncthreads();
  const int t = tsh;
  for (int j = threadIdx.x; j < m0; j += NTHR) sm[d.oSig + j] = sig[j];
  const double s0 = sig[0];
  for (int idx = threadIdx.x; idx < m0 * t; idx += NTHR) {
    const int i = idx % m0, j = idx / m0;
    const bool ok = s0 > 0.0 && sig[j] > 1e-13 * s0;
    sm[d.oCoef + i + j * d.MA] = ok ? B[i + perm[j] * LDA] / (sig[j] * sig[j]) : 0.0;
  }
  for (int j = threadIdx.x; j < t; j += NTHR) sm[d.oFill + j] = (s0 > 0.0 && sig[j] > 1e-13 * s0) ? 0.0 : 1.0;
}

void launch_aug_svd(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  hipLaunchKernelGGL(s_aug_svd, dim3(nsd), dim3(NTHR), 0, st, d, axis, sd0);
}

// ---------------------------------------------------------------- Cholesky QR

// One pass of (shifted, optionally pivoted) Cholesky QR of X = Q R: G = sum
// of partials (n x n), optional shift 11 (rows n + n (n+1)) u tr(G) (Fukaya
// et al., shifted CholeskyQR; first tried unshifted, see below),
// G[perm, perm] = R^T R (R upper triangular, or
// the symmetric square root when G is within 1e-3 of the identity), and
//   Rinv slot: P R^{-1} (rows permuted back, scaled by bscale) for the next
//              tall-skinny product Q = X P R^{-1},
//   fill slot: the mask of numerically dependent columns of Q,
//   Racc slot: the running factor with X = Q Racc -- acc_mode 1 starts it
//              with R P^T, acc_mode 2 left-multiplies it by R -- with the rows
//              of dependent columns zeroed.
// Slots have leading dimension ld.  With sout set (acc_mode 2 only), the
// transposed final factor Racc^T, zero-padded to R x R, is also stored as the
// subdomain's coefficient matrix (the S of X = Q S^T).
// skip_mode 1 (a middle pass) records in the skip slot whether this pass took
// the near-identity factor: its series remainder is below 3e-16, so its
// output is orthonormal to rounding, and the next, last pass (skip_mode 2)
// takes R = I without reading its Gram -- Rinv = bscale I, Racc unchanged --
// while its product, if it only re-orthonormalises in place, exits at once.
template <int NMAX>
__global__ __launch_bounds__(NTHR) void s_chol(Dev d, int axis, int sd0, int ndim, int rows, int ngp, int shift,
                                              int acc_mode, double bscale, int pivot, int oRinv, int oRacc, int ld,
                                              double* sout, int skip_mode) {
  const int s = sd0 + blockIdx.x;
  const int n = dim_of(d, s, axis, ndim);
  if (skip_mode == 2 && small_of(d, s)[d.oSkip] != 0.0) {
    double* sm = small_of(d, s);
    for (int idx = threadIdx.x; idx < n * n; idx += NTHR) {
      const int i = idx % n, j = idx / n;
      sm[oRinv + i + j * ld] = i == j ? bscale : 0.0;
    }
    for (int j = threadIdx.x; j < n; j += NTHR) sm[d.oFill + j] = 0.0;
    if (sout != nullptr) {
      const int R = d.R;
      double* Sg = sout + (int64_t)s * R * R;
      for (int idx = threadIdx.x; idx < R * R; idx += NTHR) {
        const int i = idx % R, j = idx / R;
        const double v = (i < n && j < n) ? sm[oRacc + j + i * ld] : 0.0;
        Sg[idx] = v;
        if (!isfinite(v)) atomicOr(d.flags, FLAG_NONFINITE);
      }
    }
    return;
  }
  __shared__ double G[LDA * CAP];
  __shared__ double X[LDA * CAP];
  __shared__ double E2[LDA * CAP];
  __shared__ double E3[LDA * CAP];
  __shared__ int dep[CAP];
  __shared__ int perm[CAP];
  __shared__ int retry;
  sum_partials(d, s, ngp, 0, n, n, n, G, LDA, 1.0);
  // the shift 11 (rows n + n (n+1)) u tr(G), every wavefront forming the
  // trace itself
  auto add_shift = [&]() {
    const int lane = threadIdx.x & 63;
    const double tr = wave_sum(lane < n ? G[lane * (LDA + 1)] : 0.0);
    const double sh = 11.0 * ((double)rows * n + (double)n * (n + 1)) * U_ROUND * tr;
    __syncthreads();
    if (threadIdx.x < n) G[threadIdx.x * (LDA + 1)] += sh;
    __syncthreads();
  };
  // The shifted pass is first tried without its shift: a Gram that is not
  // too ill-conditioned factors as it is, and the next pass then starts near
  // the identity (orthogonality error about cond(X)^2 u instead of the
  // shift's O(1)).  When a column keeps less than 1e-12 of its diagonal (or
  // is flagged dependent), the shifted factorisation is done instead.
  const bool try_plain = shift != 0;
  // A Gram within 1e-3 (Frobenius) of the identity -- the last pass of a
  // Cholesky QR, whose input is already orthonormal up to rounding, or a
  // pass over a nearly orthonormal input -- takes the symmetric factor
  // instead of the triangular one: with E = G - I, the binomial series
  //   R    = G^(1/2)  = I + E/2 - E^2/8 + E^3/16 - 5 E^4/128 ...,
  //   R^-1 = G^(-1/2) = I - E/2 + 3 E^2/8 - 5 E^3/16 + 35 E^4/128 ...,
  // cut after E^2 when |E| <= 1e-5 (remainder 0.3 |E|^3 <= 3e-16) and after
  // E^4 otherwise (remainder 0.25 |E|^5 <= 2.5e-16); R R^-1 = I to the same
  // order, and any R with G = R^T R gives an orthonormal Q = X R^-1.
  int near_order = 0;
  double fro2 = 1.0;
  if (!pivot && !shift) {
    __shared__ double red[NTHR];
    double part = 0.0;
    for (int idx = threadIdx.x; idx < n * n; idx += NTHR) {
      const int i = idx % n, j = idx / n;
      const double e = G[i + j * LDA] - (i == j ? 1.0 : 0.0);
      X[i + j * LDA] = e;  // E, kept for the near-identity factor
      part = fma(e, e, part);
    }
    fro2 = block_sum(part, red);
    near_order = fro2 <= 1e-10 ? 2 : (fro2 <= 1e-6 ? 4 : 0);
  }
  if (skip_mode == 1 && threadIdx.x == 0) small_of(d, s)[d.oSkip] = near_order > 0 ? 1.0 : 0.0;
  double* sm0 = small_of(d, s);
  if (near_order > 0) {
    // X = E from the test above (block_sum's barriers made it visible)
    mm(E2, LDA, X, LDA, false, X, LDA, false, n, n, n, 1.0, 0.0);  // E^2
    const bool o4 = near_order == 4;
    if (o4) {
      mm(E3, LDA, X, LDA, false, E2, LDA, false, n, n, n, 1.0, 0.0);  // E^3
      mm(G, LDA, E2, LDA, false, E2, LDA, false, n, n, n, 1.0, 0.0);  // E^4
    }
    for (int idx = threadIdx.x; idx < n * n; idx += NTHR) {
      const int i = idx % n, j = idx / n;
      const int o = i + j * LDA;
      const double e = X[o], e2 = E2[o], id = i == j ? 1.0 : 0.0;
      double r = id + 0.5 * e - 0.125 * e2, ri = id - 0.5 * e + 0.375 * e2;
      if (o4) {
        const double e3 = E3[o], e4 = G[o];
        r += 0.0625 * e3 - 0.0390625 * e4;
        ri += -0.3125 * e3 + 0.2734375 * e4;
      }
      G[o] = r;
      X[o] = ri;
      // outputs of the symmetric factor (no pivoting, no dependent columns)
      sm0[oRinv + i + j * ld] = bscale * ri;
    }
    for (int k = threadIdx.x; k < n; k += NTHR) {
      perm[k] = k;
      dep[k] = 0;
      sm0[d.oFill + k] = 0.0;
    }
    __syncthreads();
  } else if (try_plain) {
    for (int idx = threadIdx.x; idx < n * n; idx += NTHR) {
      const int i = idx % n, j = idx / n;
      E3[i + j * LDA] = G[i + j * LDA];
    }
    if (threadIdx.x == 0) retry = 0;
    __syncthreads();
    if (pivot) chol_inv_wave<NMAX, true>(d, G, X, n, perm, dep, E2);
    else chol_inv_wave<NMAX, false>(d, G, X, n, perm, dep, E2);
    for (int k = threadIdx.x; k < n; k += NTHR) {
      const double r = G[k * (LDA + 1)];
      if (dep[k] || !(r * r >= 1e-12 * E3[perm[k] * (LDA + 1)])) retry = 1;
    }
    __syncthreads();
    if (retry) {
      for (int idx = threadIdx.x; idx < n * n; idx += NTHR) {
        const int i = idx % n, j = idx / n;
        G[i + j * LDA] = E3[i + j * LDA];
      }
      __syncthreads();
      add_shift();
      if (pivot) chol_inv_wave<NMAX, true>(d, G, X, n, perm, dep, E2);
      else chol_inv_wave<NMAX, false>(d, G, X, n, perm, dep, E2);
    }
  } else if (pivot) {
    chol_inv_wave<NMAX, true>(d, G, X, n, perm, dep, E2);
  } else {
    chol_inv_wave<NMAX, false>(d, G, X, n, perm, dep, E2);
  }
  double* sm = sm0;
  // thread (column c = tid % 64, rows i = tid / 64 mod 4) for the n x n outputs
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  if (near_order == 0) {
    // P R^{-1}: row i of R^{-1} becomes row perm[i]
    if (c < n)
      for (int i = g; i < n; i += 4) sm[oRinv + perm[i] + c * ld] = bscale * X[i + c * LDA];
    for (int j = threadIdx.x; j < n; j += NTHR) sm[d.oFill + j] = dep[j] ? 1.0 : 0.0;
    // rows of dependent columns do not contribute to X = Q R
    if (c < n)
      for (int i = g; i < n; i += 4)
        if (dep[i]) G[i + c * LDA] = 0.0;
    __syncthreads();
  }
  if (acc_mode == 1) {
    // Racc = R P^T: column c of R becomes column perm[c]
    if (c < n) {
      const int pc = perm[c];
      for (int i = g; i < n; i += 4) sm[oRacc + i + pc * ld] = G[i + c * LDA];
    }
  } else if (acc_mode == 2) {
    // Racc <- R Racc, with Racc staged in LDS
    copy_to_lds(X, sm + oRacc, ld, n, n);
    if (sout == nullptr) {
      mm(sm + oRacc, ld, G, LDA, false, X, LDA, false, n, n, n, 1.0, 0.0);
    } else {
      mm(E2, LDA, G, LDA, false, X, LDA, false, n, n, n, 1.0, 0.0);
      copy_from_lds(sm + oRacc, ld, E2, n, n, 1.0);
      const int R = d.R;
      double* Sg = sout + (int64_t)s * R * R;
      for (int idx = threadIdx.x; idx < R * R; idx += NTHR) {
        const int i = idx % R, j = idx / R;
        const double v = (i < n && j < n) ? E2[j + i * LDA] : 0.0;
        Sg[idx] = v;
        if (!isfinite(v)) atomicOr(d.flags, FLAG_NONFINITE);
      }
    }
  }
}

void launch_chol(const Dev& d, int axis, int sd0, int nsd, int ndim, int rows, int ngp, bool shift, int acc_mode,
                 double bscale, bool pivot, int oRinv, int oRacc, int ld, hipStream_t st, double* sout, int skip_mode) {
  const int cap = ndim == DIM_M0 ? d.MA : (ndim == DIM_T ? d.T : d.R);
#define DD_CHOL(NMAX)                                                                                             \
  hipLaunchKernelGGL(s_chol<NMAX>, dim3(nsd), dim3(NTHR), 0, st, d, axis, sd0, ndim, rows, ngp, shift ? 1 : 0,   \
                     acc_mode, bscale, pivot ? 1 : 0, oRinv, oRacc, ld, sout, skip_mode)
  if (cap <= 16) DD_CHOL(16);
  else if (cap <= 32) DD_CHOL(32);
  else if (cap <= 48) DD_CHOL(48);
  else DD_CHOL(64);
#undef DD_CHOL
}

// ---------------------------------------------------------------- advection

// |C| = sign(C) C for a symmetric C (t x t in LDS, ld LDA), left in Y:
// then C+ = (C + |C|) / 2 = P diag(max(lam, 0)) P^T and C- = (C - |C|) / 2
// without the eigenvectors.  sign(C) by the scaled Newton-Schulz iteration
// (Chen and Chow, 2014): X0 = C / |C|_F has its eigenvalues in
// [-1, -l] u [l, 1], and
//   X <- a X (3 I - a^2 X^2) / 2,  a = sqrt(3 / (1 + l + l^2)),
// maps that set into [-1, -l'] u [l', 1] with l' = a l (3 - a^2 l^2) / 2
// (about 2.6 l while l is small, then quadratic convergence).  The scaled
// phase starts from l = 1e-4 / sqrt(t) (about 15 iterations); each step maps
// [0, l] monotonically into [0, l'], so eigenvalues below that bound end it
// somewhere in (0, 1) with their sign, and the unscaled iteration
// X <- X (3 I - X^2) / 2 (at most 48 steps) then carries them to +-1 until
// an update changes X by at most 1e-14 in Frobenius norm; exactly zero
// eigenvalues stay zero.  A component still moving by less than that is at
// most 2e-14 |C|_F, and so is its error in C+-.  Two products of order
// 16 NT per iteration on the FP64 matrix cores, NK k steps of 4 each.  C is
// zero-padded to order 16 NT in place; X, Y and W are LDS work buffers of
// the same shape.
template <int NT, int NK>
__device__ void abs_split(double* C, double* X, double* Y, double* W, int t) {
  constexpr int NP = 16 * NT;
  __shared__ double red[NTHR];
  double part = 0.0;
  for (int idx = threadIdx.x; idx < NP * NP; idx += NTHR) {
    const int i = idx % NP, j = idx / NP;
    const double c = (i < t && j < t) ? C[i + j * LDA] : 0.0;
    part = fma(c, c, part);
  }
  const double fro = sqrt(block_sum(part, red));
  const double ifro = fro > 0.0 ? 1.0 / fro : 0.0;
  for (int idx = threadIdx.x; idx < NP * NP; idx += NTHR) {
    const int i = idx % NP, j = idx / NP;
    const double c = (i < t && j < t) ? C[i + j * LDA] : 0.0;
    C[i + j * LDA] = c;
    X[i + j * LDA] = c * ifro;
  }
  __syncthreads();
  double l = 1e-4 / sqrt((double)t);
  for (int it = 0; it < 64 && 1.0 - l > 1e-15; ++it) {
    const double a2 = 3.0 / (1.0 + l + l * l), a = sqrt(a2);
    const double c1 = 1.5 * a, c3 = -0.5 * a * a2;
    sym_mm<NT, NK>(Y, X, X, 1.0, 0.0, Y);  // X^2
    sym_mm<NT, NK>(W, X, Y, c3, c1, X);    // c1 X + c3 X^3
    double* sw = X;
    X = W;
    W = sw;
    l = l * (c1 + c3 * l * l);
  }
  for (int it = 0; it < 48; ++it) {
    sym_mm<NT, NK>(Y, X, X, 1.0, 0.0, Y);    // X^2
    sym_mm<NT, NK>(W, X, Y, -0.5, 1.5, X);   // (3 X - X^3) / 2
    double ch = 0.0;
    for (int idx = threadIdx.x; idx < NP * NP; idx += NTHR) {
      const int o = idx % NP + (idx / NP) * LDA;
      const double dlt = W[o] - X[o];
      ch = fma(dlt, dlt, ch);
    }
    const double ch2 = block_sum(ch, red);
    double* sw = X;
    X = W;
    W = sw;
    if (ch2 <= 1e-28) break;
  }
  sym_mm<NT, NK>(Y, X, C, 1.0, 0.0, Y);  // sign(C) C
}

// Angular Galerkin matrices -> the upwind split C = C+ + C- of Appendix A
// (C = P diag(lam) P^T, C+ = P diag(max(lam,0)) P^T, C- = P diag(min(lam,0))
// P^T), and the
// coefficient matrices of the fused K-step (with nu = dt c / h, Am = S T):
//   M0 = Am (I - nu C+ + nu C-), Mm = nu Am C+, Mp = -nu Am C-,
//   GLo = nu Am En C+, GHi = -nu Am Ep C-,
//   GLoN = nu S_lo Olo C+, GHiN = -nu S_hi Ohi C-.
__global__ __launch_bounds__(NTHR) void s_adv_prep(Dev d, int axis, int sd0) {
  const int s = sd0 + blockIdx.x;
  const int lo = neighbour(d, s, axis, -1), hi = neighbour(d, s, axis, +1);
  const int r = d.rank[s], rl = lo >= 0 ? d.rank[lo] : 0, rh = hi >= 0 ? d.rank[hi] : 0;
  const int t = d.tdim[s];
  const int R = d.R, T = d.T;
  double* sm = small_of(d, s);
  __shared__ double A[LDA * CAP];
  __shared__ double Xb[LDA * CAP];
  const int pT = 0, pC = R * T, pEp = pC + T * T, pEn = pEp + T * T, pOlo = pEn + T * T, pOhi = pOlo + R * T;
  {
    const PartBlock blk[6] = {{pT, R, r, t, sm + d.oTm, R, 1.0},      {pEp, t, t, t, sm + d.oEp, T, 1.0},
                              {pEn, t, t, t, sm + d.oEn, T, 1.0},     {pOlo, R, rl, t, sm + d.oOlo, R, 1.0},
                              {pOhi, R, rh, t, sm + d.oOhi, R, 1.0},  {pC, t, t, t, A, LDA, 1.0}};
    sum_partials_blocks<6>(d, s, d.nwgM, blk);
  }
  // symmetrise C (the partial sums are symmetric up to rounding order)
  for (int idx = threadIdx.x; idx < t * t; idx += NTHR) {
    const int i = idx % t, j = idx / t;
    if (i < j) {
      const double v = 0.5 * (A[i + j * LDA] + A[j + i * LDA]);
      A[i + j * LDA] = v;
      A[j + i * LDA] = v;
    }
  }
  __syncthreads();
  // C+ and C- without the eigenvectors (see abs_split)
  __shared__ double X2[LDA * CAP];
  __shared__ double Xn[LDA * CAP];
  // tiles of 16 and k steps of 4 (an even number) covering t
  switch ((t + 7) >> 3) {
    case 1: abs_split<1, 2>(A, Xb, X2, Xn, t); break;
    case 2: abs_split<1, 4>(A, Xb, X2, Xn, t); break;
    case 3: abs_split<2, 6>(A, Xb, X2, Xn, t); break;
    case 4: abs_split<2, 8>(A, Xb, X2, Xn, t); break;
    case 5: abs_split<3, 10>(A, Xb, X2, Xn, t); break;
    case 6: abs_split<3, 12>(A, Xb, X2, Xn, t); break;
    case 7: abs_split<4, 14>(A, Xb, X2, Xn, t); break;
    default: abs_split<4, 16>(A, Xb, X2, Xn, t); break;
  }
  double* Cp = sm + d.oCp;
  double* Cn = sm + d.oCn;
  for (int idx = threadIdx.x; idx < t * t; idx += NTHR) {
    const int i = idx % t, j = idx / t;
    const double c = A[i + j * LDA], ab = 0.5 * (X2[i + j * LDA] + X2[j + i * LDA]);
    Cp[i + j * T] = 0.5 * (c + ab);
    Cn[i + j * T] = 0.5 * (c - ab);
  }
  __syncthreads();
  const double nu = d.dt * d.c / d.h;
  const double* Sg = d.S + (int64_t)s * R * R;
  double* Am = sm + d.oAm;
  mm(Am, R, Sg, R, false, sm + d.oTm, R, false, r, t, r, 1.0, 0.0);
  double* W1 = sm + d.oW1;
  double* W2 = sm + d.oW2;
  double* W3 = sm + d.oW3;
  mm(W1, R, Am, R, false, Cp, T, false, r, t, t, 1.0, 0.0);  // Am C+
  mm(W2, R, Am, R, false, Cn, T, false, r, t, t, 1.0, 0.0);  // Am C-
  for (int idx = threadIdx.x; idx < r * t; idx += NTHR) {
    const int i = idx % r, j = idx / r;
    const int o = i + j * R;
    sm[d.oM0 + o] = Am[o] - nu * W1[o] + nu * W2[o];
    sm[d.oMm + o] = nu * W1[o];
    sm[d.oMp + o] = -nu * W2[o];
  }
  __syncthreads();
  mm(W3, T, sm + d.oEn, T, false, Cp, T, false, t, t, t, 1.0, 0.0);  // En C+
  mm(sm + d.oGLo, R, Am, R, false, W3, T, false, r, t, t, nu, 0.0);
  mm(W3, T, sm + d.oEp, T, false, Cn, T, false, t, t, t, 1.0, 0.0);  // Ep C-
  mm(sm + d.oGHi, R, Am, R, false, W3, T, false, r, t, t, -nu, 0.0);
  if (rl > 0) {
    mm(W1, R, sm + d.oOlo, R, false, Cp, T, false, rl, t, t, 1.0, 0.0);
    mm(sm + d.oGLoN, R, d.S + (int64_t)lo * R * R, R, false, W1, R, false, rl, t, rl, nu, 0.0);
  }
  if (rh > 0) {
    mm(W2, R, sm + d.oOhi, R, false, Cn, T, false, rh, t, t, 1.0, 0.0);
    mm(sm + d.oGHiN, R, d.S + (int64_t)hi * R * R, R, false, W2, R, false, rh, t, rh, -nu, 0.0);
  }
}

void launch_adv_prep(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  hipLaunchKernelGGL(s_adv_prep, dim3(nsd), dim3(NTHR), 0, st, d, axis, sd0);
}

// S-step (eq. advx_evolS, integrated with the opposite sign) and the L-step
// coefficients.  With Q = h U^1 and the frozen boundary data
//   BKlo = Q[lo face]^T K^b_lo,  K^b_lo = U[lo face] Am En + U_lo[hi face] S_lo Olo,
//   BKhi = Q[hi face]^T K^b_hi,  K^b_hi = U[hi face] Am Ep + U_hi[lo face] S_hi Ohi,
//   H-(S) = Gm S - BKlo,  H+(S) = Gp S + BKhi,
//   S1 = h Racc,  S2 = S1 + dt c (H-(S1) C+ + H+(S1) C-),
// and P0 = S2^T, Pm = -dt c H-(S2)^T, Pp = -dt c H+(S2)^T for the L-step.
__global__ __launch_bounds__(NTHR) void s_adv_sstep(Dev d, int axis, int sd0) {
  const int s = sd0 + blockIdx.x;
  const int lo = neighbour(d, s, axis, -1), hi = neighbour(d, s, axis, +1);
  const int r = d.rank[s], rl = lo >= 0 ? d.rank[lo] : 0, rh = hi >= 0 ? d.rank[hi] : 0;
  const int t = d.tdim[s];
  const int R = d.R, T = d.T;
  double* sm = small_of(d, s);
  const double ih = 1.0 / d.h;
  double* Gm = sm + d.oGm;
  double* Gp = sm + d.oGp;
  // Galerkin matrices and the face products, summed from the
  // spatial-reduction partials in one pass
  double* Xlo = sm + d.oW1;  // t x r
  double* Xhi = sm + d.oW2;  // t x r
  double* Xln = sm + d.oW3;  // t x rl
  double* Xhn = sm + d.oW4;  // t x rh
  const int oX = 2 * T * T;
  {
    const PartBlock blk[5] = {{0, t, t, t, Gp, T, ih},
                              {oX, T, t, r, Xlo, T, 1.0},
                              {oX + T * R, T, t, r, Xhi, T, 1.0},
                              {oX + 2 * T * R, T, t, rl, Xln, T, 1.0},
                              {oX + 3 * T * R, T, t, rh, Xhn, T, 1.0}};
    sum_partials_blocks<5>(d, s, d.nwgN, blk);
  }
  double* W5 = sm + d.oW5;
  double* W6 = sm + d.oW6;
  double* BKlo = sm + d.oBKlo;
  double* BKhi = sm + d.oBKhi;
  double* S1 = sm + d.oS1;
  double* S2 = sm + d.oS2;
  // independent products share a pass (mm_multi); S1 and S2 serve as
  // scratch until they are formed
  //   BKlo = Xlo (Am En) + Xln (S_lo Olo),  BKhi = Xhi (Am Ep) + Xhn (S_hi Ohi)
  const double* Slo = lo >= 0 ? d.S + (int64_t)lo * R * R : d.S;
  const double* Shi = hi >= 0 ? d.S + (int64_t)hi * R * R : d.S;
  {
    const MMOp ops[4] = {{W5, R, sm + d.oAm, R, false, sm + d.oEn, T, false, r, t, t, 1.0, 0.0, W5, R},
                         {S1, T, sm + d.oAm, R, false, sm + d.oEp, T, false, r, t, t, 1.0, 0.0, S1, T},
                         {W6, R, Slo, R, false, sm + d.oOlo, R, false, rl, t, rl, 1.0, 0.0, W6, R},
                         {S2, T, Shi, R, false, sm + d.oOhi, R, false, rh, t, rh, 1.0, 0.0, S2, T}};
    mm_multi(ops);
  }
  {
    const MMOp ops[2] = {{BKlo, T, Xlo, T, false, W5, R, false, t, t, r, 1.0, 0.0, BKlo, T},
                         {BKhi, T, Xhi, T, false, S1, T, false, t, t, r, 1.0, 0.0, BKhi, T}};
    mm_multi(ops);
  }
  {
    const MMOp ops[2] = {{BKlo, T, Xln, T, false, W6, R, false, t, t, rl, 1.0, 1.0, BKlo, T},
                         {BKhi, T, Xhn, T, false, S2, T, false, t, t, rh, 1.0, 1.0, BKhi, T}};
    mm_multi(ops);
  }
  // S1 = h Racc; Gm = -Gp^T (the spatial reduction forms Gp only)
  for (int idx = threadIdx.x; idx < t * t; idx += NTHR) {
    const int i = idx % t, j = idx / t;
    S1[i + j * T] = d.h * sm[d.oRacc + i + j * T];
    Gm[i + j * T] = -Gp[j + i * T];
  }
  __syncthreads();
  double* Hm = sm + d.oW5;
  double* Hp = sm + d.oW6;
  {
    const MMOp ops[2] = {{Hm, T, Gm, T, false, S1, T, false, t, t, t, 1.0, 0.0, Hm, T},
                         {Hp, T, Gp, T, false, S1, T, false, t, t, t, 1.0, 0.0, Hp, T}};
    mm_multi(ops);
  }
  for (int idx = threadIdx.x; idx < t * t; idx += NTHR) {
    const int o = (idx % t) + (idx / t) * T;
    Hm[o] -= BKlo[o];
    Hp[o] += BKhi[o];
    S2[o] = S1[o];
  }
  __syncthreads();
  const double dc = d.dt * d.c;
  mm(S2, T, Hm, T, false, sm + d.oCp, T, false, t, t, t, dc, 1.0);
  mm(S2, T, Hp, T, false, sm + d.oCn, T, false, t, t, t, dc, 1.0);
  {
    const MMOp ops[2] = {{Hm, T, Gm, T, false, S2, T, false, t, t, t, 1.0, 0.0, Hm, T},
                         {Hp, T, Gp, T, false, S2, T, false, t, t, t, 1.0, 0.0, Hp, T}};
    mm_multi(ops);
  }
  for (int idx = threadIdx.x; idx < t * t; idx += NTHR) {
    const int i = idx % t, j = idx / t;
    const int o = i + j * T, ot = j + i * T;
    sm[d.oP0 + ot] = S2[o];
    sm[d.oPm + ot] = -dc * (Hm[o] - BKlo[o]);
    sm[d.oPp + ot] = -dc * (Hp[o] + BKhi[o]);
  }
}

void launch_adv_sstep(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  hipLaunchKernelGGL(s_adv_sstep, dim3(nsd), dim3(NTHR), 0, st, d, axis, sd0);
}

// Truncation (Algorithm 5) of S3 = RL^T: SVD through two Jacobi passes on
// Gram matrices (S3^T S3, then (S3 Y1)^T (S3 Y1)), rank rule, and the
// rotations Bu = U~[:, :r'] / h, Bv = V~[:, :r'] for the final products.
// Writes S = diag(sigma[:r']) into the state and r' into rnew.  With
// fold_rinv, the last Cholesky-QR product of L is folded into the rotation:
// Bv = Rinv V~[:, :r'] with Rinv the last pass's inverse factor, so that
// V = X2 Bv / sqrt(w) straight from the second-pass output X2.
__global__ __launch_bounds__(NTHR) void s_trunc(Dev d, int axis, int sd0, int fold_rinv) {
  const int s = sd0 + blockIdx.x;
  const int t = d.tdim[s];
  const int R = d.R, T = d.T;
  double* sm = small_of(d, s);
  __shared__ double G[LDA * CAP];
  __shared__ double Y[LDA * CAP];
  __shared__ double sig[CAP];
  __shared__ int perm[CAP];
  __shared__ int rsh;
  __shared__ double red[NTHR];
  __shared__ double sv[CAP];
  __shared__ int anyfill;
  const double* RL = sm + d.oRacc;
  double* Ut = sm + d.oW4;   // t x r'
  // B = S3 = RL^T; one-sided Jacobi: S3 V = U Sigma
  for (int idx = threadIdx.x; idx < t * t; idx += NTHR) {
    const int i = idx % t, j = idx / t;
    G[i + j * LDA] = RL[j + i * T];
  }
  __syncthreads();
  jacobi_1s(d, G, t, t, Y, 1e-14, 1e-15, 40);
  col_norms(G, t, t, sv);
  sort_desc(sv, t, perm);
  for (int j = threadIdx.x; j < t; j += NTHR) sig[j] = sv[perm[j]];
  __syncthreads();
  if (threadIdx.x == 0) {
    int rp;
    const int cap = min(min(d.r_max, t), R);
    if (d.forced && d.force[2 * d.nsub + axis * d.nsub + s] > 0) {
      rp = min(d.force[2 * d.nsub + axis * d.nsub + s], min(t, R));
    } else if (d.rank_mode == 0) {
      rp = min(d.r_fixed, min(t, R));
    } else {
      rp = max(d.r_min, tail_rank(sig, t, d.tol));
      if (rp > cap) {
        rp = cap;
        atomicAdd(d.clamps, 1ull);
        if (d.strict) atomicOr(d.flags, FLAG_RANK_CLAMP);
      }
    }
    if (rp < 1) rp = 1;
    rsh = rp;
    d.rnew[s] = rp;
    anyfill = 0;
  }
  __syncthreads();
  const int rp = rsh;
  for (int idx = threadIdx.x; idx < t * rp; idx += NTHR) {
    const int i = idx % t, j = idx / t;
    sm[d.oBv + i + j * T] = Y[i + perm[j] * LDA];
  }
  // U~ = S3 V / sigma (pseudo-random where sigma vanishes)
  const double s0 = sig[0];
  for (int idx = threadIdx.x; idx < t * rp; idx += NTHR) {
    const int i = idx % t, j = idx / t;
    double v;
    if (s0 > 0.0 && sig[j] > 1e-13 * s0) {
      v = G[i + perm[j] * LDA] / sig[j];
    } else {
      v = hash_unit(((uint64_t)s << 40) ^ ((uint64_t)(j + 1000) << 24) ^ (uint64_t)i);
      anyfill = 1;
    }
    Ut[i + j * T] = v;
  }
  __syncthreads();
  // completed columns are made orthonormal to the others (two passes of
  // modified Gram-Schmidt); the Jacobi columns already are
  if (anyfill) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int j = 0; j < rp; ++j) {
        for (int k = 0; k < j; ++k) {
          double part = 0.0;
          for (int i = threadIdx.x; i < t; i += NTHR) part = fma(Ut[i + k * T], Ut[i + j * T], part);
          red[threadIdx.x] = part;
          __syncthreads();
          for (int off = NTHR / 2; off > 0; off >>= 1) {
            if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
            __syncthreads();
          }
          const double dot = red[0];
          __syncthreads();
          for (int i = threadIdx.x; i < t; i += NTHR) Ut[i + j * T] -= dot * Ut[i + k * T];
          __syncthreads();
        }
        double part = 0.0;
        for (int i = threadIdx.x; i < t; i += NTHR) part = fma(Ut[i + j * T], Ut[i + j * T], part);
        red[threadIdx.x] = part;
        __syncthreads();
        for (int off = NTHR / 2; off > 0; off >>= 1) {
          if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
          __syncthreads();
        }
        const double nrm = sqrt(red[0]);
        __syncthreads();
        const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
        for (int i = threadIdx.x; i < t; i += NTHR) Ut[i + j * T] *= inv;
        __syncthreads();
      }
    }
  }
  const double ih = 1.0 / d.h;
  for (int idx = threadIdx.x; idx < t * rp; idx += NTHR) {
    const int i = idx % t, j = idx / t;
    sm[d.oBu + i + j * T] = Ut[i + j * T] * ih;
  }
  double* Sg = d.S + (int64_t)s * R * R;
  for (int idx = threadIdx.x; idx < R * R; idx += NTHR) {
    const int i = idx % R, j = idx / R;
    const double v = (i == j && i < rp) ? sig[i] : 0.0;
    Sg[idx] = v;
  }
  if (threadIdx.x < rp && !isfinite(sig[threadIdx.x])) atomicOr(d.flags, FLAG_NONFINITE);
  if (fold_rinv) {
    // G is free again; the barriers above ordered the Bv stores
    __syncthreads();
    mm(G, LDA, sm + d.oRinv, T, false, sm + d.oBv, T, false, t, rp, t, 1.0, 0.0);
    copy_from_lds(sm + d.oBv, T, G, t, rp, 1.0);
  }
}

void launch_trunc(const Dev& d, int axis, int sd0, int nsd, bool fold_rinv, hipStream_t st) {
  hipLaunchKernelGGL(s_trunc, dim3(nsd), dim3(NTHR), 0, st, d, axis, sd0, fold_rinv ? 1 : 0);
}

// ---------------------------------------------------------------- collision

// m = V^T w (the angular averages <V_j>, eq. coll_evolK): every thread
// accumulates all r sums over its directions, then r threads add the
// NTHR partials in a fixed order.
__global__ __launch_bounds__(NTHR) void s_coll_prep(Dev d, int sd0) {
  const int s = sd0 + blockIdx.x;
  const int r = d.rank[s];
  const int M = d.M, R = d.R;
  __shared__ double red[CAPR * NTHR];
  const double* Vs = d.V + (int64_t)s * M * R;
  double acc[CAPR];
#pragma unroll
  for (int a = 0; a < CAPR; ++a) acc[a] = 0.0;
  for (int q = threadIdx.x; q < M; q += NTHR) {
    const double wq = d.w[q];
#pragma unroll
    for (int a = 0; a < CAPR; ++a)
      if (a < r) acc[a] = fma(Vs[(int64_t)a * M + q], wq, acc[a]);
  }
#pragma unroll
  for (int a = 0; a < CAPR; ++a)
    if (a < r) red[a * NTHR + threadIdx.x] = acc[a];
  __syncthreads();
  if (threadIdx.x < r) {
    double sum = 0.0;
    for (int k = 0; k < NTHR; ++k) sum += red[threadIdx.x * NTHR + k];
    small_of(d, s)[d.oMv + threadIdx.x] = sum;
  }
}

void launch_coll_prep(const Dev& d, int sd0, int nsd, hipStream_t st) {
  hipLaunchKernelGGL(s_coll_prep, dim3(nsd), dim3(NTHR), 0, st, d, sd0);
}

// S-step (eq. coll_evolS) and L-step coefficients (eq. coll_evolL):
//   S2 = S1 + dt (-(1/W) Gs S1 m m^T + Gt S1 - q m^T),  S1 = h Racc,
//   P = S2^T (I - dt Gt),  crow = dt ((S2 m)^T Gs / W + q^T).
// All operands are staged in LDS (leading dimension L, the stored-rank
// capacity: 21, or 64 in the wide plan).
// The collision S- and L-steps with RK4 substeps (nested form: four stages
// out = base + alpha f(in), alpha = dt/4, dt/3, dt/2, dt).
//   S-step: f(S) = -(1/W) Gs S m m^T + Gt S - q m^T, from S1;
//   L-step: L = V N + 1 y^T stays of that form, with
//           f(N, y) = (-N Gt, (1/W) Gs N^T m + (Gs - Gt) y + q), from (S2^T, 0);
// the result gives P = N and Crow = y for the L-step product L1 = V P + 1 Crow^T.
// Stage buffers of order r: S2 (LDS) and the small workspace slots W1, W2.
template <int L>
__device__ void coll_sstep_rk4(const Dev& d, int s, int r, const double* Gs, const double* Gt, const double* S1,
                               double* S2, const double* qv, const double* mv, double* v1, double* v2, double* v3) {
  const int T = d.T, R = d.R;
  const double iW = 1.0 / d.W;
  double* sm = small_of(d, s);
  double* Xg = sm + d.oW1;
  double* Yg = sm + d.oW2;
  for (int stg = 0; stg < 4; ++stg) {
    const double al = d.dt / (double)(4 - stg);
    // Sin = S1 (LDS, ld L) at the first stage, else Xg (ld T)
    const double* Sin = stg == 0 ? S1 : Xg;
    const int ldi = stg == 0 ? L : T;
    for (int i = threadIdx.x; i < r; i += NTHR) {
      double acc = 0.0;
      for (int k = 0; k < r; ++k) acc = fma(Sin[i + k * ldi], mv[k], acc);
      v1[i] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < r; i += NTHR) {
      double acc = 0.0;
      for (int k = 0; k < r; ++k) acc = fma(Gs[i + k * L], v1[k], acc);
      v2[i] = acc;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < r * r; idx += NTHR) {
      const int i = idx % r, j = idx / r;
      double g = 0.0;
      for (int k = 0; k < r; ++k) g = fma(Gt[i + k * L], Sin[k + j * ldi], g);
      S2[i + j * L] = S1[i + j * L] + al * (-iW * v2[i] * mv[j] + g - qv[i] * mv[j]);
    }
    __syncthreads();
    if (stg < 3) {
      for (int idx = threadIdx.x; idx < r * r; idx += NTHR) {
        const int i = idx % r, j = idx / r;
        Xg[i + j * T] = S2[i + j * L];
      }
      __syncthreads();
    }
  }
  // L-step: (N, y) from (S2^T, 0); stage inputs in Xg / Yg alternately, y in v3
  for (int i = threadIdx.x; i < r; i += NTHR) v3[i] = 0.0;
  __syncthreads();
  for (int stg = 0; stg < 4; ++stg) {
    const double al = d.dt / (double)(4 - stg);
    double* Nout = (stg & 1) ? Yg : Xg;
    const double* Nin = (stg & 1) ? Xg : Yg;  // unused at the first stage
    // v1 = N_in^T m, then v2 = y_out
    for (int j = threadIdx.x; j < r; j += NTHR) {
      double acc = 0.0;
      for (int k = 0; k < r; ++k) acc = fma(stg == 0 ? S2[j + k * L] : Nin[k + j * T], mv[k], acc);
      v1[j] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < r; i += NTHR) {
      double a = 0.0, b = 0.0;
      for (int k = 0; k < r; ++k) {
        a = fma(Gs[i + k * L], v1[k], a);
        b = fma(Gs[i + k * L] - Gt[i + k * L], v3[k], b);
      }
      v2[i] = al * (iW * a + b + qv[i]);
    }
    for (int idx = threadIdx.x; idx < r * r; idx += NTHR) {
      const int i = idx % r, j = idx / r;
      double g = 0.0;
      for (int k = 0; k < r; ++k) g = fma(stg == 0 ? S2[k + i * L] : Nin[i + k * T], Gt[k + j * L], g);
      Nout[i + j * T] = S2[j + i * L] - al * g;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < r; i += NTHR) v3[i] = v2[i];
    __syncthreads();
  }
  // the last stage (odd) wrote Yg
  for (int idx = threadIdx.x; idx < r * r; idx += NTHR) {
    const int i = idx % r, j = idx / r;
    sm[d.oP0 + i + j * R] = Yg[i + j * T];
  }
  for (int j = threadIdx.x; j < r; j += NTHR) sm[d.oCrow + j] = v3[j];
}

template <int L>
__global__ __launch_bounds__(NTHR) void s_coll_sstep(Dev d, int sd0) {
  const int s = sd0 + blockIdx.x;
  const int r = d.rank[s];
  const int R = d.R, T = d.T;
  double* sm = small_of(d, s);
  __shared__ double Gs[L * L], Gt[L * L], S1[L * L], S2[L * L];
  __shared__ double qv[L], mv[L], v1[L], v2[L], v3[L];
  {
    const PartBlock blk[3] = {{0, R, r, r, Gs, L, 1.0}, {R * R, R, r, r, Gt, L, 1.0}, {2 * R * R, R, r, 1, qv, L, 1.0}};
    sum_partials_blocks<3>(d, s, d.nwgN, blk);
  }
  for (int idx = threadIdx.x; idx < r * r; idx += NTHR) {
    const int i = idx % r, j = idx / r;
    S1[i + j * L] = d.h * sm[d.oRacc + i + j * T];
  }
  for (int i = threadIdx.x; i < r; i += NTHR) mv[i] = sm[d.oMv + i];
  __syncthreads();
  for (int i = threadIdx.x; i < r; i += NTHR) {
    double acc = 0.0;
    for (int k = 0; k < r; ++k) acc = fma(S1[i + k * L], mv[k], acc);
    v1[i] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < r; i += NTHR) {
    double acc = 0.0;
    for (int k = 0; k < r; ++k) acc = fma(Gs[i + k * L], v1[k], acc);
    v2[i] = acc;
  }
  const double dt = d.dt, iW = 1.0 / d.W;
  if (d.rk4) {
    coll_sstep_rk4<L>(d, s, r, Gs, Gt, S1, S2, qv, mv, v1, v2, v3);
    return;
  }
  mm(S2, L, Gt, L, false, S1, L, false, r, r, r, 1.0, 0.0);
  for (int idx = threadIdx.x; idx < r * r; idx += NTHR) {
    const int i = idx % r, j = idx / r;
    const int o = i + j * L;
    S2[o] = S1[o] + dt * (-iW * v2[i] * mv[j] + S2[o] - qv[i] * mv[j]);
  }
  __syncthreads();
  // P = S2^T (I - dt Gt)
  for (int idx = threadIdx.x; idx < r * r; idx += NTHR) {
    const int i = idx % r, j = idx / r;
    double acc = S2[j + i * L];
    for (int k = 0; k < r; ++k) acc = fma(-dt * S2[k + i * L], Gt[k + j * L], acc);
    sm[d.oP0 + i + j * R] = acc;
  }
  for (int i = threadIdx.x; i < r; i += NTHR) {
    double acc = 0.0;
    for (int k = 0; k < r; ++k) acc = fma(S2[i + k * L], mv[k], acc);
    v3[i] = acc;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < r; j += NTHR) {
    double acc = 0.0;
    for (int i = 0; i < r; ++i) acc = fma(v3[i], Gs[i + j * L], acc);
    sm[d.oCrow + j] = dt * (acc * iW + qv[j]);
  }
}

void launch_coll_sstep(const Dev& d, int sd0, int nsd, hipStream_t st) {
  if (d.R <= CAPR) hipLaunchKernelGGL(s_coll_sstep<CAPR>, dim3(nsd), dim3(NTHR), 0, st, d, sd0);
  else hipLaunchKernelGGL(s_coll_sstep<64>, dim3(nsd), dim3(NTHR), 0, st, d, sd0);
}

}  // namespace dd
