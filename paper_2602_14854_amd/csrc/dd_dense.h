// Dense FP64 building blocks for one workgroup (NTHR threads) working on
// small matrices in LDS: one-sided Jacobi SVD / eigensolver, Cholesky,
// triangular inverse, products, sorting and the tail rank rule.
#pragma once

#include "dd_internal.h"

namespace dd {

constexpr int LDA = CAP + 1;                        // padded leading dimension of LDS matrices
constexpr double U_ROUND = 1.1102230246251565e-16;  // 2^-53

// sum of v over the workgroup (red: NTHR doubles of LDS scratch)
__device__ inline double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = NTHR / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}


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

// sum over aligned groups of G lanes (G = 1, 2, 4, 8 or 16) with DPP
template <int G>
__device__ inline double group_sum_dpp(double v) {
  if (G == 1) return v;
  union { double d; int i[2]; } a, b;
  a.d = v;
  // quad_perm [1,0,3,2]: partner lane ^ 1
  b.i[0] = __builtin_amdgcn_update_dpp(0, a.i[0], 0xB1, 0xF, 0xF, false);
  b.i[1] = __builtin_amdgcn_update_dpp(0, a.i[1], 0xB1, 0xF, 0xF, false);
  a.d += b.d;
  if (G == 2) return a.d;
  // quad_perm [2,3,0,1]: partner lane ^ 2
  b.i[0] = __builtin_amdgcn_update_dpp(0, a.i[0], 0x4E, 0xF, 0xF, false);
  b.i[1] = __builtin_amdgcn_update_dpp(0, a.i[1], 0x4E, 0xF, 0xF, false);
  a.d += b.d;
  if (G == 4) return a.d;
  // row_half_mirror: lane i <-> 7 - i inside each group of 8 (quads are uniform)
  b.i[0] = __builtin_amdgcn_update_dpp(0, a.i[0], 0x141, 0xF, 0xF, false);
  b.i[1] = __builtin_amdgcn_update_dpp(0, a.i[1], 0x141, 0xF, 0xF, false);
  a.d += b.d;
  if (G == 8) return a.d;
  // row_mirror: lane i <-> 15 - i inside each row of 16
  b.i[0] = __builtin_amdgcn_update_dpp(0, a.i[0], 0x140, 0xF, 0xF, false);
  b.i[1] = __builtin_amdgcn_update_dpp(0, a.i[1], 0x140, 0xF, 0xF, false);
  a.d += b.d;
  return a.d;
}

// Plane rotation that orthogonalises two columns with squared norms al, be
// and inner product ga (ga != 0):  t = tan(theta) =
// 2 ga sign(be - al) / (|be - al| + hypot(be - al, 2 ga)), c = 1/sqrt(1+t^2),
// s = c t.  The square roots and the reciprocal use the hardware
// approximations followed by two Newton steps each (each step squares the
// relative error, so an initial 2^-22 reaches working precision).
__device__ inline double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = r * fma(-0.5 * x * r, r, 1.5);
  return r * fma(-0.5 * x * r, r, 1.5);
}

__device__ inline double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = r * fma(-x, r, 2.0);
  return r * fma(-x, r, 2.0);
}

__device__ inline void jacobi_rotation(double al, double be, double ga, double& c, double& sn) {
  const double df = be - al;
  const double h2 = fma(df, df, 4.0 * ga * ga);
  const double hyp = h2 * rsqrt_nr(h2);
  const double t = (df >= 0.0 ? 2.0 * ga : -2.0 * ga) * rcp_nr(fabs(df) + hyp);
  c = rsqrt_nr(fma(t, t, 1.0));
  sn = c * t;
}

// One-sided (Hestenes) Jacobi on the columns of B (rows x n, LDS, ld LDA):
// plane rotations from the right make the columns of B mutually orthogonal;
// the same rotations accumulate in V (n x n, LDS, ld LDA), so that on exit
// B_out = B_in V with orthogonal columns.  For an SVD B_in = U Sigma V^T the
// column norms are the singular values; for a positive definite B_in the
// columns of V are its eigenvectors and the norms its eigenvalues.
// Column pairs are taken in round-robin rounds; each pair is owned by a group
// of g lanes (a power of two inside one wavefront) that reduce the three
// inner products with shuffles, so a round needs a single barrier.  A pair is
// rotated while |b_p . b_q| > tol ||b_p|| ||b_q||; the relative test gives
// the small singular values of graded matrices to high relative accuracy.
// Columns whose norm is below floor_rel ||B||_F carry only rounding noise
// (a rank-deficient B) and are not rotated: rotating noise against large
// columns would keep it from ever meeting the relative test.
template <int GMAX>
__device__ int jacobi_1s_g(const Dev& d, double* B, int rows, int n, double* V, double tol, double floor_rel,
                           int max_sweeps) {
  __shared__ int rotated;
  __shared__ double red[NTHR];
  double part = 0.0;
  for (int idx = threadIdx.x; idx < rows * n; idx += NTHR) {
    const double x = B[idx % rows + (idx / rows) * LDA];
    part = fma(x, x, part);
  }
  const double floor2 = floor_rel * floor_rel * block_sum(part, red);
  for (int idx = threadIdx.x; idx < n * n; idx += NTHR) {
    const int i = idx % n, j = idx / n;
    V[i + j * LDA] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (n <= 1) return 0;
  const int n2 = n + (n & 1);
  const int npair = n2 / 2;
  const int nm1 = n2 - 1;
  constexpr int g = GMAX;
  const int grp = threadIdx.x / g, lane = threadIdx.x % g;
  const double tol2 = tol * tol;
  bool converged = false;
  int sweeps = 0;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    sweeps = sweep + 1;
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    // round-robin positions: position 0 is fixed, positions 1..n2-1 rotate
    int va = grp - 1, vb = n2 - 2 - grp;  // (position - 1 + round), kept below nm1
    for (int round = 0; round < nm1; ++round) {
      {
        const int a = grp == 0 ? 0 : va + 1;
        const int b = vb + 1;
        const int p = a < b ? a : b, q = a < b ? b : a;
        const bool live = grp < npair && q < n;
        double al = 0.0, be = 0.0, ga = 0.0;
        if (live) {
          for (int i = lane; i < rows; i += g) {
            const double x = B[i + p * LDA], y = B[i + q * LDA];
            al = fma(x, x, al);
            be = fma(y, y, be);
            ga = fma(x, y, ga);
          }
        }
        {
          al = group_sum_dpp<GMAX>(al);
          be = group_sum_dpp<GMAX>(be);
          ga = group_sum_dpp<GMAX>(ga);
          if (live && ga != 0.0 && al > floor2 && be > floor2 && ga * ga > tol2 * al * be) {
            double c, sn;
            jacobi_rotation(al, be, ga, c, sn);
            for (int i = lane; i < rows; i += g) {
              const double x = B[i + p * LDA], y = B[i + q * LDA];
              B[i + p * LDA] = c * x - sn * y;
              B[i + q * LDA] = fma(sn, x, c * y);
            }
            for (int i = lane; i < n; i += g) {
              const double x = V[i + p * LDA], y = V[i + q * LDA];
              V[i + p * LDA] = c * x - sn * y;
              V[i + q * LDA] = fma(sn, x, c * y);
            }
            if (lane == 0) rotated = 1;
          }
        }
      }
      if (++va >= nm1) va -= nm1;
      if (++vb >= nm1) vb -= nm1;
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) {
      converged = true;
      break;
    }
  }
  if (!converged && tol < 1e-12 && threadIdx.x == 0) atomicOr(d.flags, FLAG_JACOBI_NOCONV);
  __syncthreads();
  return converged ? sweeps : -sweeps;
}

// One-sided Jacobi with the default lane-group size.
__device__ inline int jacobi_1s(const Dev& d, double* B, int rows, int n, double* V, double tol, double floor_rel,
                                int max_sweeps) {
  const int npair = (n + (n & 1)) / 2;
  if (npair * 16 <= NTHR) return jacobi_1s_g<16>(d, B, rows, n, V, tol, floor_rel, max_sweeps);
  return jacobi_1s_g<8>(d, B, rows, n, V, tol, floor_rel, max_sweeps);
}

// norms of the columns of B (rows x n, LDS) into out[n]
__device__ void col_norms(const double* B, int rows, int n, double* out) {
  for (int j = threadIdx.x; j < n; j += NTHR) {
    double acc = 0.0;
    for (int i = 0; i < rows; ++i) acc = fma(B[i + j * LDA], B[i + j * LDA], acc);
    out[j] = sqrt(acc);
  }
  __syncthreads();
}

// perm[j] = index of the j-th largest of vals[0..n) (ties keep index order)
__device__ void sort_desc(const double* vals, int n, int* perm) {
  for (int j = threadIdx.x; j < n; j += NTHR) {
    const double v = vals[j];
    int rank = 0;
    for (int k = 0; k < n; ++k) {
      const double w = vals[k];
      rank += (w > v || (w == v && k < j)) ? 1 : 0;
    }
    perm[rank] = j;
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

// X = R^{-1} for upper triangular R (both LDS, ld LDA): back substitution of
// R X = I row by row from the bottom, each row eliminated from the rows
// above in parallel (two barriers per row).
__device__ void tri_inv_upper(const double* R, double* X, int n) {
  for (int idx = threadIdx.x; idx < n * n; idx += NTHR) {
    const int i = idx % n, j = idx / n;
    X[i + j * LDA] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = n - 1; k >= 0; --k) {
    const double ir = 1.0 / R[k + k * LDA];
    for (int j = k + threadIdx.x; j < n; j += NTHR) X[k + j * LDA] *= ir;
    __syncthreads();
    const int w = n - k;
    for (int idx = threadIdx.x; idx < k * w; idx += NTHR) {
      const int i = idx % k, j = k + idx / k;
      X[i + j * LDA] = fma(-R[i + k * LDA], X[k + j * LDA], X[i + j * LDA]);
    }
    __syncthreads();
  }
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

}  // namespace dd
