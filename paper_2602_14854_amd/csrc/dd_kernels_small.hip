// Small dense FP64 kernels of the DD-DLRA step: one workgroup per subdomain
// works on matrices of at most 64 x 64 (the intermediate rank t or the
// augmentation width m0).  They add the tall-skinny kernels' partial sums in
// a fixed order, run the serial linear algebra (two-sided Jacobi
// eigensolver, Cholesky, triangular inverse) and form the coefficient
// matrices of the next tall-skinny pass.
#include "dd_internal.h"

namespace dd {

constexpr int LDA = CAP + 1;        // padded leading dimension of LDS matrices
constexpr int CAPR = 21;
constexpr double U_ROUND = 1.1102230246251565e-16;  // 2^-53

// ---------------------------------------------------------------- helpers

// C (m x n) = alpha * op(A) op(B) (+ beta C); generic pointers, no aliasing.
__device__ void mm(double* C, int ldc, const double* A, int lda, bool ta, const double* B, int ldb,
                   bool tb, int m, int n, int k, double alpha, double beta) {
  for (int idx = threadIdx.x; idx < m * n; idx += NTHR) {
    const int i = idx % m, j = idx / m;
    double acc = 0.0;
    for (int l = 0; l < k; ++l) {
      const double a = ta ? A[l + i * lda] : A[i + l * lda];
      const double b = tb ? B[j + l * ldb] : B[l + j * ldb];
      acc = fma(a, b, acc);
    }
    C[i + j * ldc] = (beta == 0.0) ? alpha * acc : alpha * acc + beta * C[i + j * ldc];
  }
  __syncthreads();
}

// dst (rows x cols, ldd) = sum over ngp workgroup partials of the block at
// offset off (leading dimension lds) -- fixed order, deterministic.
__device__ void sum_partials(const Dev& d, int s, int ngp, int off, int lds, int rows, int cols, double* dst,
                             int ldd, double scale) {
  const double* gp = gpart_of(d, s);
  for (int idx = threadIdx.x; idx < rows * cols; idx += NTHR) {
    const int i = idx % rows, j = idx / rows;
    double acc = 0.0;
    for (int w = 0; w < ngp; ++w) acc += gp[(int64_t)w * d.gpTile + off + i + j * lds];
    dst[i + j * ldd] = scale * acc;
  }
  __syncthreads();
}

// Cyclic two-sided Jacobi on the symmetric n x n matrix A (LDS, ld LDA),
// parallel over disjoint pairs with the round-robin ordering.  On exit the
// diagonal of A holds the eigenvalues and Y (ld LDA) the eigenvectors.
// rel = true: a rotation is skipped when |a_pq| <= 1e-15 sqrt(|a_pp a_qq|),
// which gives eigenvalues of positive definite graded matrices to high
// relative accuracy; rel = false uses 1e-15 ||A||_F.
__device__ void jacobi_eig(const Dev& d, double* A, double* Y, int n, bool rel) {
  __shared__ double cs[CAP];
  __shared__ int pq[CAP];
  __shared__ int rotated;
  __shared__ double fro;
  for (int idx = threadIdx.x; idx < n * n; idx += NTHR) {
    const int i = idx % n, j = idx / n;
    Y[i + j * LDA] = (i == j) ? 1.0 : 0.0;
  }
  if (threadIdx.x == 0) {
    double f = 0.0;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) f += A[i + j * LDA] * A[i + j * LDA];
    fro = sqrt(f);
  }
  __syncthreads();
  if (n <= 1) return;
  const int n2 = n + (n & 1);
  const int npair = n2 / 2;
  const double atol = 1e-15 * fro;
  bool converged = false;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < n2 - 1; ++round) {
      if (threadIdx.x < npair) {
        const int k = threadIdx.x;
        const int pa = k, pb = n2 - 1 - k;
        const int a = pa == 0 ? 0 : ((pa - 1 + round) % (n2 - 1)) + 1;
        const int b = ((pb - 1 + round) % (n2 - 1)) + 1;
        const int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, sn = 0.0;
        if (q < n) {
          const double app = A[p + p * LDA], aqq = A[q + q * LDA], apq = A[p + q * LDA];
          const double thr = rel ? 1e-15 * sqrt(fabs(app * aqq)) : atol;
          if (fabs(apq) > thr && apq != 0.0) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double at = fabs(tau);
            const double tt = (at > 1e150) ? 0.5 / tau : copysign(1.0, tau) / (at + sqrt(1.0 + at * at));
            c = 1.0 / sqrt(1.0 + tt * tt);
            sn = tt * c;
            rotated = 1;
          }
        }
        cs[2 * k] = c;
        cs[2 * k + 1] = sn;
        pq[2 * k] = p;
        pq[2 * k + 1] = q;
      }
      __syncthreads();
      for (int idx = threadIdx.x; idx < npair * n; idx += NTHR) {
        const int k = idx / n, j = idx % n;
        const double sn = cs[2 * k + 1];
        if (sn == 0.0) continue;
        const double c = cs[2 * k];
        const int p = pq[2 * k], q = pq[2 * k + 1];
        const double ap = A[p + j * LDA], aq = A[q + j * LDA];
        A[p + j * LDA] = c * ap - sn * aq;
        A[q + j * LDA] = sn * ap + c * aq;
      }
      __syncthreads();
      for (int idx = threadIdx.x; idx < npair * n; idx += NTHR) {
        const int k = idx / n, i = idx % n;
        const double sn = cs[2 * k + 1];
        if (sn == 0.0) continue;
        const double c = cs[2 * k];
        const int p = pq[2 * k], q = pq[2 * k + 1];
        const double ap = A[i + p * LDA], aq = A[i + q * LDA];
        A[i + p * LDA] = c * ap - sn * aq;
        A[i + q * LDA] = sn * ap + c * aq;
        const double yp = Y[i + p * LDA], yq = Y[i + q * LDA];
        Y[i + p * LDA] = c * yp - sn * yq;
        Y[i + q * LDA] = sn * yp + c * yq;
      }
      __syncthreads();
      if (threadIdx.x < npair && cs[2 * threadIdx.x + 1] != 0.0) {
        const int p = pq[2 * threadIdx.x], q = pq[2 * threadIdx.x + 1];
        A[p + q * LDA] = 0.0;
        A[q + p * LDA] = 0.0;
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) {
      converged = true;
      break;
    }
  }
  if (!converged && threadIdx.x == 0) atomicOr(d.flags, FLAG_JACOBI_NOCONV);
  __syncthreads();
}

// descending order of the diagonal of A: perm[j] = index of the j-th largest
__device__ void sort_desc(const double* A, int n, int* perm) {
  if (threadIdx.x == 0) {
    for (int j = 0; j < n; ++j) perm[j] = j;
    for (int j = 0; j < n; ++j) {
      int best = j;
      for (int k = j + 1; k < n; ++k)
        if (A[perm[k] + perm[k] * LDA] > A[perm[best] + perm[best] * LDA]) best = k;
      const int tmp = perm[j];
      perm[j] = perm[best];
      perm[best] = tmp;
    }
  }
  __syncthreads();
}

// In-place upper Cholesky of the n x n matrix G (LDS, ld LDA): G = R^T R.
// A pivot that is not larger than 1e-20 times the column's own diagonal
// entry means the column is numerically dependent on the earlier ones (the
// matrix being factored is rank-deficient).  Such a pivot is set to 1 so the
// factorisation continues as if the column were a fresh unit direction, and
// dep[k] is set: the caller replaces that column by a pseudo-random vector
// and zeroes the row in the accumulated R, which keeps A = Q R exact up to
// the dependent column's residual.  A non-finite pivot latches
// FLAG_NONFINITE.
__device__ void chol_upper(const Dev& d, double* G, int n, int* dep) {
  __shared__ double diag0[CAP];
  for (int i = threadIdx.x; i < n; i += NTHR) {
    diag0[i] = G[i + i * LDA];
    dep[i] = 0;
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      double dk = G[k + k * LDA];
      if (!isfinite(dk)) {
        atomicOr(d.flags, FLAG_NONFINITE);
        dk = 1.0;
        dep[k] = 1;
      } else if (!(dk > 1e-20 * diag0[k])) {
        dk = 1.0;
        dep[k] = 1;
      }
      G[k + k * LDA] = sqrt(dk);
    }
    __syncthreads();
    const double rkk = G[k + k * LDA];
    for (int j = k + 1 + threadIdx.x; j < n; j += NTHR) G[k + j * LDA] /= rkk;
    for (int i = k + 1 + threadIdx.x; i < n; i += NTHR) G[i + k * LDA] = 0.0;
    __syncthreads();
    const int m = n - k - 1;
    for (int idx = threadIdx.x; idx < m * m; idx += NTHR) {
      const int i = k + 1 + idx % m, j = k + 1 + idx / m;
      if (i <= j) G[i + j * LDA] -= G[k + i * LDA] * G[k + j * LDA];
    }
    __syncthreads();
  }
}

// X = R^{-1} for upper triangular R (both LDS, ld LDA)
__device__ void tri_inv_upper(const double* R, double* X, int n) {
  for (int j = threadIdx.x; j < n; j += NTHR) {
    for (int i = n - 1; i > j; --i) X[i + j * LDA] = 0.0;
    X[j + j * LDA] = 1.0 / R[j + j * LDA];
    for (int i = j - 1; i >= 0; --i) {
      double acc = 0.0;
      for (int k = i + 1; k <= j; ++k) acc = fma(R[i + k * LDA], X[k + j * LDA], acc);
      X[i + j * LDA] = -acc / R[i + i * LDA];
    }
  }
  __syncthreads();
}

// smallest k with (sum_{j >= k} sig_j^2)^(1/2) <= tol (Algorithms 4, 5)
__device__ int tail_rank(const double* sig, int n, double tol) {
  double tail2 = 0.0;
  int k = n;
  for (int j = n - 1; j >= 0; --j) {
    tail2 += sig[j] * sig[j];
    if (sqrt(tail2) <= tol) k = j;
    else break;
  }
  return k;
}

__device__ void copy_to_lds(double* dst, const double* src, int lds, int rows, int cols) {
  for (int idx = threadIdx.x; idx < rows * cols; idx += NTHR) {
    const int i = idx % rows, j = idx / rows;
    dst[i + j * LDA] = src[i + j * lds];
  }
  __syncthreads();
}

__device__ void copy_from_lds(double* dst, int ldd, const double* src, int rows, int cols, double scale) {
  for (int idx = threadIdx.x; idx < rows * cols; idx += NTHR) {
    const int i = idx % rows, j = idx / rows;
    dst[i + j * ldd] = scale * src[i + j * LDA];
  }
  __syncthreads();
}

// ---------------------------------------------------------------- augmentation

// First pass of the weighted SVD of L0 (Algorithm 4, step 2): eigenvectors of
// the Gram matrix A^T A, A = sqrt(w) L0.
__global__ __launch_bounds__(NTHR) void s_aug_eig1(Dev d, int axis, int sd0) {
  const int s = sd0 + blockIdx.x;
  const int m0 = m0_of(d, s, axis);
  __shared__ double G[LDA * CAP];
  __shared__ double Y[LDA * CAP];
  sum_partials(d, s, d.nwgM, 0, m0, m0, m0, G, LDA, 1.0);
  jacobi_eig(d, G, Y, m0, true);
  copy_from_lds(small_of(d, s) + d.oY1, d.MA, Y, m0, m0, 1.0);
}

void launch_aug_eig1(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  hipLaunchKernelGGL(s_aug_eig1, dim3(nsd), dim3(NTHR), 0, st, d, axis, sd0);
}

// Second pass: Gram of Z = A Y1 (nearly diagonal, so Jacobi resolves small
// singular values to relative accuracy), singular values, the rank rule of
// Algorithm 4 step 3, and the coefficients of V-hat = Z Y2[:, :t] / sigma.
__global__ __launch_bounds__(NTHR) void s_aug_eig2(Dev d, int axis, int sd0) {
  const int s = sd0 + blockIdx.x;
  const int m0 = m0_of(d, s, axis);
  const int r = d.rank[s];
  __shared__ double G[LDA * CAP];
  __shared__ double Y[LDA * CAP];
  __shared__ double sig[CAP];
  __shared__ int perm[CAP];
  __shared__ int tsh;
  sum_partials(d, s, d.nwgM, 0, m0, m0, m0, G, LDA, 1.0);
  jacobi_eig(d, G, Y, m0, true);
  sort_desc(G, m0, perm);
  for (int j = threadIdx.x; j < m0; j += NTHR) sig[j] = sqrt(fmax(G[perm[j] + perm[j] * LDA], 0.0));
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
  double* sm = small_of(d, s);
  for (int j = threadIdx.x; j < m0; j += NTHR) sm[d.oSig + j] = sig[j];
  const double s0 = sig[0];
  for (int idx = threadIdx.x; idx < m0 * t; idx += NTHR) {
    const int i = idx % m0, j = idx / m0;
    const bool ok = s0 > 0.0 && sig[j] > 1e-13 * s0;
    sm[d.oCoef + i + j * d.MA] = ok ? Y[i + perm[j] * LDA] / sig[j] : 0.0;
  }
  for (int j = threadIdx.x; j < t; j += NTHR) sm[d.oFill + j] = (s0 > 0.0 && sig[j] > 1e-13 * s0) ? 0.0 : 1.0;
}

void launch_aug_eig2(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  hipLaunchKernelGGL(s_aug_eig2, dim3(nsd), dim3(NTHR), 0, st, d, axis, sd0);
}

// ---------------------------------------------------------------- Cholesky QR

// One pass of (shifted) Cholesky QR: G = sum of partials (n x n), optional
// shift 11 (rows n + n (n+1)) u tr(G) (Fukaya et al., shifted CholeskyQR),
// R = chol(G), Rinv = bscale R^{-1} for the next tall-skinny product, the
// fill mask of numerically dependent columns, and the running product of R
// factors (acc_mode 1: start, 2: left-multiply) with the dependent rows
// zeroed.
__global__ __launch_bounds__(NTHR) void s_chol(Dev d, int axis, int sd0, int ndim, int rows, int ngp, int shift,
                                              int acc_mode, double bscale) {
  const int s = sd0 + blockIdx.x;
  const int n = dim_of(d, s, axis, ndim);
  __shared__ double G[LDA * CAP];
  __shared__ double X[LDA * CAP];
  __shared__ int dep[CAP];
  sum_partials(d, s, ngp, 0, n, n, n, G, LDA, 1.0);
  if (shift) {
    if (threadIdx.x == 0) {
      double tr = 0.0;
      for (int i = 0; i < n; ++i) tr += G[i + i * LDA];
      const double sh = 11.0 * ((double)rows * n + (double)n * (n + 1)) * U_ROUND * tr;
      for (int i = 0; i < n; ++i) G[i + i * LDA] += sh;
    }
    __syncthreads();
  }
  chol_upper(d, G, n, dep);
  tri_inv_upper(G, X, n);
  double* sm = small_of(d, s);
  copy_from_lds(sm + d.oRinv, d.T, X, n, n, bscale);
  for (int j = threadIdx.x; j < n; j += NTHR) sm[d.oFill + j] = dep[j] ? 1.0 : 0.0;
  // rows of dependent columns do not contribute to A = Q R
  for (int idx = threadIdx.x; idx < n * n; idx += NTHR) {
    const int i = idx % n, j = idx / n;
    if (dep[i]) G[i + j * LDA] = 0.0;
  }
  __syncthreads();
  if (acc_mode == 1) {
    copy_from_lds(sm + d.oRacc, d.T, G, n, n, 1.0);
  } else if (acc_mode == 2) {
    // X = G * Racc (upper x upper), then store
    const double* Ra = sm + d.oRacc;
    for (int idx = threadIdx.x; idx < n * n; idx += NTHR) {
      const int i = idx % n, j = idx / n;
      double acc = 0.0;
      for (int k = i; k <= j; ++k) acc = fma(G[i + k * LDA], Ra[k + j * d.T], acc);
      X[i + j * LDA] = (i <= j) ? acc : 0.0;
    }
    __syncthreads();
    copy_from_lds(sm + d.oRacc, d.T, X, n, n, 1.0);
  }
}

void launch_chol(const Dev& d, int axis, int sd0, int nsd, int ndim, int rows, int ngp, bool shift, int acc_mode,
                 double bscale, hipStream_t st) {
  hipLaunchKernelGGL(s_chol, dim3(nsd), dim3(NTHR), 0, st, d, axis, sd0, ndim, rows, ngp, shift ? 1 : 0, acc_mode,
                     bscale);
}

// ---------------------------------------------------------------- advection

// Angular Galerkin matrices -> eigen-split C = P diag(lam) P^T (Appendix A),
// C+ = P diag(max(lam,0)) P^T, C- = P diag(min(lam,0)) P^T, and the
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
  __shared__ double P[LDA * CAP];
  __shared__ double lam[CAP];
  const int pT = 0, pC = R * T, pEp = pC + T * T, pEn = pEp + T * T, pOlo = pEn + T * T, pOhi = pOlo + R * T;
  sum_partials(d, s, d.nwgM, pT, R, r, t, sm + d.oTm, R, 1.0);
  sum_partials(d, s, d.nwgM, pEp, t, t, t, sm + d.oEp, T, 1.0);
  sum_partials(d, s, d.nwgM, pEn, t, t, t, sm + d.oEn, T, 1.0);
  if (rl > 0) sum_partials(d, s, d.nwgM, pOlo, R, rl, t, sm + d.oOlo, R, 1.0);
  if (rh > 0) sum_partials(d, s, d.nwgM, pOhi, R, rh, t, sm + d.oOhi, R, 1.0);
  sum_partials(d, s, d.nwgM, pC, t, t, t, A, LDA, 1.0);
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
  jacobi_eig(d, A, P, t, false);
  for (int j = threadIdx.x; j < t; j += NTHR) lam[j] = A[j + j * LDA];
  __syncthreads();
  double* Cp = sm + d.oCp;
  double* Cn = sm + d.oCn;
  for (int idx = threadIdx.x; idx < t * t; idx += NTHR) {
    const int i = idx % t, j = idx / t;
    double ap = 0.0, an = 0.0;
    for (int k = 0; k < t; ++k) {
      const double pp = P[i + k * LDA] * P[j + k * LDA];
      ap = fma(pp, fmax(lam[k], 0.0), ap);
      an = fma(pp, fmin(lam[k], 0.0), an);
    }
    Cp[i + j * T] = ap;
    Cn[i + j * T] = an;
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
__global__ __launch_bounds__(NTHR) void s_adv_sstep(Dev d, int axis, int sd0, const double* Qb) {
  const int s = sd0 + blockIdx.x;
  const int lo = neighbour(d, s, axis, -1), hi = neighbour(d, s, axis, +1);
  const int r = d.rank[s], rl = lo >= 0 ? d.rank[lo] : 0, rh = hi >= 0 ? d.rank[hi] : 0;
  const int t = d.tdim[s];
  const int N = d.N, R = d.R, T = d.T;
  double* sm = small_of(d, s);
  const double ih = 1.0 / d.h;
  double* Gm = sm + d.oGm;
  double* Gp = sm + d.oGp;
  sum_partials(d, s, d.nwgN, 0, t, t, t, Gm, T, ih);
  sum_partials(d, s, d.nwgN, T * T, t, t, t, Gp, T, ih);
  // face products
  const double* Q = Qb + (int64_t)s * N * T;
  const double* Us = d.U + (int64_t)s * N * R;
  const double* Ul = lo >= 0 ? d.U + (int64_t)lo * N * R : nullptr;
  const double* Uh = hi >= 0 ? d.U + (int64_t)hi * N * R : nullptr;
  const int nf = face_len(d, axis);
  double* Xlo = sm + d.oW1;  // t x r
  double* Xhi = sm + d.oW2;  // t x r
  double* Xln = sm + d.oW3;  // t x rl
  double* Xhn = sm + d.oW4;  // t x rh
  const int ntot = t * r * 2 + t * rl + t * rh;
  for (int e = threadIdx.x; e < ntot; e += NTHR) {
    int blk, ee, nc;
    if (e < t * r) { blk = 0; ee = e; nc = r; }
    else if (e < 2 * t * r) { blk = 1; ee = e - t * r; nc = r; }
    else if (e < 2 * t * r + t * rl) { blk = 2; ee = e - 2 * t * r; nc = rl; }
    else { blk = 3; ee = e - 2 * t * r - t * rl; nc = rh; }
    const int i = ee % t, c = ee / t;
    (void)nc;
    double acc = 0.0;
    for (int f = 0; f < nf; ++f) {
      const int pl = face_cell(d, axis, false, f), ph = face_cell(d, axis, true, f);
      if (blk == 0) acc = fma(Q[(int64_t)i * N + pl], Us[(int64_t)c * N + pl], acc);
      else if (blk == 1) acc = fma(Q[(int64_t)i * N + ph], Us[(int64_t)c * N + ph], acc);
      else if (blk == 2) acc = fma(Q[(int64_t)i * N + pl], Ul[(int64_t)c * N + ph], acc);
      else acc = fma(Q[(int64_t)i * N + ph], Uh[(int64_t)c * N + pl], acc);
    }
    double* dst = blk == 0 ? Xlo : blk == 1 ? Xhi : blk == 2 ? Xln : Xhn;
    dst[i + c * T] = acc;
  }
  __syncthreads();
  double* W5 = sm + d.oW5;
  double* W6 = sm + d.oW6;
  double* BKlo = sm + d.oBKlo;
  double* BKhi = sm + d.oBKhi;
  // BKlo = Xlo (Am En) + Xln (S_lo Olo)
  mm(W5, R, sm + d.oAm, R, false, sm + d.oEn, T, false, r, t, t, 1.0, 0.0);
  mm(BKlo, T, Xlo, T, false, W5, R, false, t, t, r, 1.0, 0.0);
  if (rl > 0) {
    mm(W6, R, d.S + (int64_t)lo * R * R, R, false, sm + d.oOlo, R, false, rl, t, rl, 1.0, 0.0);
    mm(BKlo, T, Xln, T, false, W6, R, false, t, t, rl, 1.0, 1.0);
  }
  mm(W5, R, sm + d.oAm, R, false, sm + d.oEp, T, false, r, t, t, 1.0, 0.0);
  mm(BKhi, T, Xhi, T, false, W5, R, false, t, t, r, 1.0, 0.0);
  if (rh > 0) {
    mm(W6, R, d.S + (int64_t)hi * R * R, R, false, sm + d.oOhi, R, false, rh, t, rh, 1.0, 0.0);
    mm(BKhi, T, Xhn, T, false, W6, R, false, t, t, rh, 1.0, 1.0);
  }
  // S1 = h Racc
  double* S1 = sm + d.oS1;
  double* S2 = sm + d.oS2;
  for (int idx = threadIdx.x; idx < t * t; idx += NTHR) {
    const int i = idx % t, j = idx / t;
    S1[i + j * T] = d.h * sm[d.oRacc + i + j * T];
  }
  __syncthreads();
  double* Hm = sm + d.oW5;
  double* Hp = sm + d.oW6;
  mm(Hm, T, Gm, T, false, S1, T, false, t, t, t, 1.0, 0.0);
  mm(Hp, T, Gp, T, false, S1, T, false, t, t, t, 1.0, 0.0);
  for (int idx = threadIdx.x; idx < t * t; idx += NTHR) {
    const int o = (idx % t) + (idx / t) * T;
    Hm[o] -= BKlo[o];
    Hp[o] += BKhi[o];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < t * t; idx += NTHR) {
    const int o = (idx % t) + (idx / t) * T;
    S2[o] = S1[o];
  }
  __syncthreads();
  const double dc = d.dt * d.c;
  mm(S2, T, Hm, T, false, sm + d.oCp, T, false, t, t, t, dc, 1.0);
  mm(S2, T, Hp, T, false, sm + d.oCn, T, false, t, t, t, dc, 1.0);
  mm(Hm, T, Gm, T, false, S2, T, false, t, t, t, 1.0, 0.0);
  mm(Hp, T, Gp, T, false, S2, T, false, t, t, t, 1.0, 0.0);
  for (int idx = threadIdx.x; idx < t * t; idx += NTHR) {
    const int i = idx % t, j = idx / t;
    const int o = i + j * T, ot = j + i * T;
    sm[d.oP0 + ot] = S2[o];
    sm[d.oPm + ot] = -dc * (Hm[o] - BKlo[o]);
    sm[d.oPp + ot] = -dc * (Hp[o] + BKhi[o]);
  }
}

void launch_adv_sstep(const Dev& d, int axis, int sd0, int nsd, const double* Q, hipStream_t st) {
  hipLaunchKernelGGL(s_adv_sstep, dim3(nsd), dim3(NTHR), 0, st, d, axis, sd0, Q);
}

// Truncation (Algorithm 5) of S3 = RL^T: SVD through two Jacobi passes on
// Gram matrices (S3^T S3, then (S3 Y1)^T (S3 Y1)), rank rule, and the
// rotations Bu = U~[:, :r'] / h, Bv = V~[:, :r'] for the final products.
// Writes S = diag(sigma[:r']) into the state and r' into rnew.
__global__ __launch_bounds__(NTHR) void s_trunc(Dev d, int axis, int sd0) {
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
  const double* RL = sm + d.oRacc;
  double* S3 = sm + d.oW1;   // t x t
  double* Z = sm + d.oW2;    // t x t
  double* Y1 = sm + d.oW3;   // t x t
  double* Ut = sm + d.oW4;   // t x r'
  for (int idx = threadIdx.x; idx < t * t; idx += NTHR) {
    const int i = idx % t, j = idx / t;
    S3[i + j * T] = RL[j + i * T];
  }
  __syncthreads();
  // pass 1: G = S3^T S3
  for (int idx = threadIdx.x; idx < t * t; idx += NTHR) {
    const int i = idx % t, j = idx / t;
    double acc = 0.0;
    for (int k = 0; k < t; ++k) acc = fma(S3[k + i * T], S3[k + j * T], acc);
    G[i + j * LDA] = acc;
  }
  __syncthreads();
  jacobi_eig(d, G, Y, t, true);
  copy_from_lds(Y1, T, Y, t, t, 1.0);
  mm(Z, T, S3, T, false, Y1, T, false, t, t, t, 1.0, 0.0);
  // pass 2: G = Z^T Z
  for (int idx = threadIdx.x; idx < t * t; idx += NTHR) {
    const int i = idx % t, j = idx / t;
    double acc = 0.0;
    for (int k = 0; k < t; ++k) acc = fma(Z[k + i * T], Z[k + j * T], acc);
    G[i + j * LDA] = acc;
  }
  __syncthreads();
  jacobi_eig(d, G, Y, t, true);
  sort_desc(G, t, perm);
  for (int j = threadIdx.x; j < t; j += NTHR) sig[j] = sqrt(fmax(G[perm[j] + perm[j] * LDA], 0.0));
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
  }
  __syncthreads();
  const int rp = rsh;
  // Bv = Y1 Y2[:, perm[:r']]
  for (int idx = threadIdx.x; idx < t * rp; idx += NTHR) {
    const int i = idx % t, j = idx / t;
    double acc = 0.0;
    for (int k = 0; k < t; ++k) acc = fma(Y1[i + k * T], Y[k + perm[j] * LDA], acc);
    sm[d.oBv + i + j * T] = acc;
  }
  // U~ = Z Y2[:, perm[:r']] / sigma (pseudo-random where sigma vanishes)
  const double s0 = sig[0];
  for (int idx = threadIdx.x; idx < t * rp; idx += NTHR) {
    const int i = idx % t, j = idx / t;
    double v;
    if (s0 > 0.0 && sig[j] > 1e-13 * s0) {
      double acc = 0.0;
      for (int k = 0; k < t; ++k) acc = fma(Z[i + k * T], Y[k + perm[j] * LDA], acc);
      v = acc / sig[j];
    } else {
      v = hash_unit(((uint64_t)s << 40) ^ ((uint64_t)(j + 1000) << 24) ^ (uint64_t)i);
    }
    Ut[i + j * T] = v;
  }
  __syncthreads();
  // two passes of modified Gram-Schmidt on U~ (t x r')
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
}

void launch_trunc(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  hipLaunchKernelGGL(s_trunc, dim3(nsd), dim3(NTHR), 0, st, d, axis, sd0);
}

__global__ void s_set_rank(Dev d, int sd0, int nsd) {
  const int s = sd0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (s < sd0 + nsd) d.rank[s] = d.rnew[s];
}

void launch_set_rank(const Dev& d, int sd0, int nsd, hipStream_t st) {
  hipLaunchKernelGGL(s_set_rank, dim3((nsd + 63) / 64), dim3(64), 0, st, d, sd0, nsd);
}

// ---------------------------------------------------------------- collision

// m = V^T w (the angular averages <V_j>, eq. coll_evolK)
__global__ __launch_bounds__(NTHR) void s_coll_prep(Dev d, int sd0) {
  const int s = sd0 + blockIdx.x;
  const int r = d.rank[s];
  const int M = d.M, R = d.R;
  __shared__ double red[NTHR];
  const double* Vs = d.V + (int64_t)s * M * R;
  double* sm = small_of(d, s);
  for (int a = 0; a < r; ++a) {
    double acc = 0.0;
    for (int q = threadIdx.x; q < M; q += NTHR) acc = fma(Vs[(int64_t)a * M + q], d.w[q], acc);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = NTHR / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) sm[d.oMv + a] = red[0];
    __syncthreads();
  }
}

void launch_coll_prep(const Dev& d, int sd0, int nsd, hipStream_t st) {
  hipLaunchKernelGGL(s_coll_prep, dim3(nsd), dim3(NTHR), 0, st, d, sd0);
}

// S-step (eq. coll_evolS) and L-step coefficients (eq. coll_evolL):
//   S2 = S1 + dt (-(1/W) Gs S1 m m^T + Gt S1 - q m^T),  S1 = h Racc,
//   P = S2^T (I - dt Gt),  crow = dt ((S2 m)^T Gs / W + q^T).
__global__ __launch_bounds__(NTHR) void s_coll_sstep(Dev d, int sd0) {
  const int s = sd0 + blockIdx.x;
  const int r = d.rank[s];
  const int R = d.R, T = d.T;
  double* sm = small_of(d, s);
  double* Gs = sm + d.oGs;
  double* Gt = sm + d.oGt;
  double* qv = sm + d.oQv;
  sum_partials(d, s, d.nwgN, 0, R, r, r, Gs, R, 1.0);
  sum_partials(d, s, d.nwgN, R * R, R, r, r, Gt, R, 1.0);
  sum_partials(d, s, d.nwgN, 2 * R * R, R, r, 1, qv, R, 1.0);
  const double* mv = sm + d.oMv;
  double* S1 = sm + d.oS1;
  double* S2 = sm + d.oS2;
  __shared__ double v1[CAPR], v2[CAPR], v3[CAPR];
  for (int idx = threadIdx.x; idx < r * r; idx += NTHR) {
    const int i = idx % r, j = idx / r;
    S1[i + j * R] = d.h * sm[d.oRacc + i + j * T];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < r; i += NTHR) {
    double acc = 0.0;
    for (int k = 0; k < r; ++k) acc = fma(S1[i + k * R], mv[k], acc);
    v1[i] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < r; i += NTHR) {
    double acc = 0.0;
    for (int k = 0; k < r; ++k) acc = fma(Gs[i + k * R], v1[k], acc);
    v2[i] = acc;
  }
  __syncthreads();
  mm(S2, R, Gt, R, false, S1, R, false, r, r, r, 1.0, 0.0);
  const double dt = d.dt, iW = 1.0 / d.W;
  for (int idx = threadIdx.x; idx < r * r; idx += NTHR) {
    const int i = idx % r, j = idx / r;
    const int o = i + j * R;
    S2[o] = S1[o] + dt * (-iW * v2[i] * mv[j] + S2[o] - qv[i] * mv[j]);
  }
  __syncthreads();
  // P = S2^T (I - dt Gt)
  for (int idx = threadIdx.x; idx < r * r; idx += NTHR) {
    const int i = idx % r, j = idx / r;
    double acc = S2[j + i * R];
    for (int k = 0; k < r; ++k) acc = fma(-dt * S2[k + i * R], Gt[k + j * R], acc);
    sm[d.oP0 + i + j * R] = acc;
  }
  for (int i = threadIdx.x; i < r; i += NTHR) {
    double acc = 0.0;
    for (int k = 0; k < r; ++k) acc = fma(S2[i + k * R], mv[k], acc);
    v3[i] = acc;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < r; j += NTHR) {
    double acc = 0.0;
    for (int i = 0; i < r; ++i) acc = fma(v3[i], Gs[i + j * R], acc);
    sm[d.oCrow + j] = dt * (acc * iW + qv[j]);
  }
}

void launch_coll_sstep(const Dev& d, int sd0, int nsd, hipStream_t st) {
  hipLaunchKernelGGL(s_coll_sstep, dim3(nsd), dim3(NTHR), 0, st, d, sd0);
}

// S = RL^T after the weighted QR of L1 (Algorithm 3, step 5)
__global__ __launch_bounds__(NTHR) void s_coll_final(Dev d, int sd0) {
  const int s = sd0 + blockIdx.x;
  const int r = d.rank[s];
  const int R = d.R, T = d.T;
  const double* sm = small_of(d, s);
  double* Sg = d.S + (int64_t)s * R * R;
  for (int idx = threadIdx.x; idx < R * R; idx += NTHR) {
    const int i = idx % R, j = idx / R;
    double v = 0.0;
    if (i < r && j < r) v = sm[d.oRacc + j + i * T];
    Sg[idx] = v;
    if (!isfinite(v)) atomicOr(d.flags, FLAG_NONFINITE);
  }
}

void launch_coll_final(const Dev& d, int sd0, int nsd, hipStream_t st) {
  hipLaunchKernelGGL(s_coll_final, dim3(nsd), dim3(NTHR), 0, st, d, sd0);
}

}  // namespace dd
