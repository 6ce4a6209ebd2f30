// Dense FP64 building blocks for one workgroup (NTHR threads) working on
// small matrices in LDS: one-sided Jacobi SVD / eigensolver, Cholesky,
// triangular inverse, products, sorting and the tail rank rule.
#pragma once

#include "dd_internal.h"

namespace dd {

constexpr int LDA = CAP + 1;                        // padded leading dimension of LDS matrices
constexpr double U_ROUND = 1.1102230246251565e-16;  // 2^-53

// sum of v over the workgroup (red: NTHR doubles of LDS scratch)
__device__ __forceinline__ double block_sum(double v, double* red) {
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
// The inner loop is unrolled so that operands in global memory are fetched
// eight at a time rather than one dependent load per step.
__device__ __forceinline__ void mm(double* C, int ldc, const double* A, int lda, bool ta, const double* B, int ldb,
                   bool tb, int m, int n, int k, double alpha, double beta) {
  for (int idx = threadIdx.x; idx < m * n; idx += NTHR) {
    const int i = idx % m, j = idx / m;
    double acc = 0.0;
#pragma unroll 8
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
// offset off (leading dimension lds) -- fixed order over the partials, so
// deterministic.  Each thread takes four entries and fetches four partials of
// each before adding, keeping 16 loads in flight.
__device__ __forceinline__ void sum_partials(const Dev& d, int s, int ngp, int off, int lds, int rows, int cols, double* dst,
                             int ldd, double scale) {
  const double* gp = gpart_of(d, s) + off;
  const int n = rows * cols;
  for (int base = threadIdx.x; base < n; base += 4 * NTHR) {
    int src[4];
    double acc[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = base + e * NTHR;
      src[e] = idx < n ? (idx % rows) + (idx / rows) * lds : -1;
      acc[e] = 0.0;
    }
    for (int w0 = 0; w0 < ngp; w0 += 4) {
      double v[4][4];
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          v[e][u] = (src[e] >= 0 && w0 + u < ngp) ? gp[(int64_t)(w0 + u) * d.gpTile + src[e]] : 0.0;
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[e] += v[e][u];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = base + e * NTHR;
      if (idx < n) dst[(idx % rows) + (idx / rows) * ldd] = scale * acc[e];
    }
  }
  __syncthreads();
}

// sum over aligned groups of G lanes (G = 1, 2, 4, 8 or 16) with DPP
template <int G>
__device__ __forceinline__ double group_sum_dpp(double v) {
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
__device__ __forceinline__ double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = r * fma(-0.5 * x * r, r, 1.5);
  return r * fma(-0.5 * x * r, r, 1.5);
}

__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = r * fma(-x, r, 2.0);
  return r * fma(-x, r, 2.0);
}

__device__ __forceinline__ void jacobi_rotation(double al, double be, double ga, double& c, double& sn) {
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
// columns of V are its eigenvectors and the norms its eigenvalues.  With
// ACCV false the rotations are not accumulated.
// Column pairs are taken in round-robin rounds; each pair is owned by a group
// of G lanes (inside one wavefront), each lane holding up to RPL rows of the
// two columns (and of the two columns of V) in registers for the whole
// round, so a round is one batch of LDS reads, three group reductions with
// DPP, the rotation and one batch of LDS writes, then a single barrier.  A
// pair is rotated while |b_p . b_q| > tol ||b_p|| ||b_q||; the relative test
// gives the small singular values of graded matrices to high relative
// accuracy.  Columns whose norm is below floor_rel ||B||_F carry only
// rounding noise (a rank-deficient B) and are not rotated: rotating noise
// against large columns would keep it from ever meeting the relative test.
// Returns the number of sweeps (negative if not converged).
template <int G, int RPL, bool ACCV>
__device__ __forceinline__ int jacobi_1s_g(const Dev& d, double* B, int rows, int n, double* V, double tol, double floor_rel,
                           int max_sweeps) {
  __shared__ int rotated[3];  // per-sweep flags: set, read, cleared in rotation
  __shared__ double red[NTHR];
  double part = 0.0;
  for (int idx = threadIdx.x; idx < rows * n; idx += NTHR) {
    const double x = B[idx % rows + (idx / rows) * LDA];
    part = fma(x, x, part);
  }
  const double floor2 = floor_rel * floor_rel * block_sum(part, red);
  if (ACCV) {
    for (int idx = threadIdx.x; idx < n * n; idx += NTHR) {
      const int i = idx % n, j = idx / n;
      V[i + j * LDA] = (i == j) ? 1.0 : 0.0;
    }
  }
  if (threadIdx.x < 3) rotated[threadIdx.x] = 0;
  __syncthreads();
  if (n <= 1) return 0;
  const int n2 = n + (n & 1);
  const int npair = n2 / 2;
  const int nm1 = n2 - 1;
  const int grp = threadIdx.x / G, lane = threadIdx.x % G;
  const double tol2 = tol * tol;
  bool converged = false;
  int sweeps = 0;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    sweeps = sweep + 1;
    const int slot = sweep % 3;
    if (threadIdx.x == 0) rotated[(sweep + 1) % 3] = 0;
    // round-robin positions: position 0 is fixed, positions 1..n2-1 rotate
    int va = grp - 1, vb = n2 - 2 - grp;  // (position - 1 + round), kept below nm1
    for (int round = 0; round < nm1; ++round) {
      const int a = grp == 0 ? 0 : va + 1;
      const int b = vb + 1;
      const int p = a < b ? a : b, q = a < b ? b : a;
      const bool live = grp < npair && q < n;
      double x[RPL], y[RPL], vx[RPL], vy[RPL];
#pragma unroll
      for (int m = 0; m < RPL; ++m) {
        const int i = lane + G * m;
        const bool in = live && i < rows;
        x[m] = in ? B[i + p * LDA] : 0.0;
        y[m] = in ? B[i + q * LDA] : 0.0;
        if (ACCV) {
          const bool inv = live && i < n;
          vx[m] = inv ? V[i + p * LDA] : 0.0;
          vy[m] = inv ? V[i + q * LDA] : 0.0;
        }
      }
      double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
      for (int m = 0; m < RPL; ++m) {
        al = fma(x[m], x[m], al);
        be = fma(y[m], y[m], be);
        ga = fma(x[m], y[m], ga);
      }
      al = group_sum_dpp<G>(al);
      be = group_sum_dpp<G>(be);
      ga = group_sum_dpp<G>(ga);
      if (live && ga != 0.0 && al > floor2 && be > floor2 && ga * ga > tol2 * al * be) {
        double c, sn;
        jacobi_rotation(al, be, ga, c, sn);
#pragma unroll
        for (int m = 0; m < RPL; ++m) {
          const int i = lane + G * m;
          if (i < rows) {
            B[i + p * LDA] = c * x[m] - sn * y[m];
            B[i + q * LDA] = fma(sn, x[m], c * y[m]);
          }
          if (ACCV && i < n) {
            V[i + p * LDA] = c * vx[m] - sn * vy[m];
            V[i + q * LDA] = fma(sn, vx[m], c * vy[m]);
          }
        }
        if (lane == 0) rotated[slot] = 1;
      }
      if (++va >= nm1) va -= nm1;
      if (++vb >= nm1) vb -= nm1;
      __syncthreads();
    }
    if (!rotated[slot]) {
      converged = true;
      break;
    }
  }
  if (!converged && tol < 1e-12 && threadIdx.x == 0) atomicOr(d.flags, FLAG_JACOBI_NOCONV);
  __syncthreads();
  return converged ? sweeps : -sweeps;
}

// One-sided Jacobi, lane groups and register rows chosen from the size:
// 16 lanes per pair up to 32 columns, else 8 (rows <= 64 either way).
__device__ __forceinline__ int jacobi_1s(const Dev& d, double* B, int rows, int n, double* V, double tol, double floor_rel,
                                int max_sweeps) {
  if (n <= 32 && rows <= 32) {
    if (V) return jacobi_1s_g<16, 2, true>(d, B, rows, n, V, tol, floor_rel, max_sweeps);
    return jacobi_1s_g<16, 2, false>(d, B, rows, n, V, tol, floor_rel, max_sweeps);
  }
  if (V) return jacobi_1s_g<8, 8, true>(d, B, rows, n, V, tol, floor_rel, max_sweeps);
  return jacobi_1s_g<8, 8, false>(d, B, rows, n, V, tol, floor_rel, max_sweeps);
}

// norms of the columns of B (rows x n, LDS) into out[n]
__device__ __forceinline__ void col_norms(const double* B, int rows, int n, double* out) {
  for (int j = threadIdx.x; j < n; j += NTHR) {
    double acc = 0.0;
    for (int i = 0; i < rows; ++i) acc = fma(B[i + j * LDA], B[i + j * LDA], acc);
    out[j] = sqrt(acc);
  }
  __syncthreads();
}

// perm[j] = index of the j-th largest of vals[0..n) (ties keep index order)
__device__ __forceinline__ void sort_desc(const double* vals, int n, int* perm) {
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

// Sum of v over the 64 lanes of a wavefront (every lane gets the total).
__device__ __forceinline__ double wave_sum(double v) {
  v = group_sum_dpp<16>(v);
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// Upper-triangle entries (i <= j) of an n x n matrix owned by this thread:
// packed index q = tid + NTHR m for m < NO.  Unused slots hold i = j = -1.
// NO = own_slots(n) suffices for an n x n matrix.
constexpr int own_slots(int n) { return (n * (n + 1) / 2 + NTHR - 1) / NTHR; }

template <int NO>
__device__ __forceinline__ void owned_pairs(int n, int* oi, int* oj) {
  const int np = n * (n + 1) / 2;
#pragma unroll
  for (int m = 0; m < NO; ++m) {
    const int q = threadIdx.x + m * NTHR;
    int i = -1, j = -1;
    if (q < np) {
      j = (int)((sqrtf(8.0f * q + 1.0f) - 1.0f) * 0.5f);
      if (j * (j + 1) / 2 > q) --j;
      if ((j + 1) * (j + 2) / 2 <= q) ++j;
      i = q - j * (j + 1) / 2;
    }
    oi[m] = i;
    oj[m] = j;
  }
}

// Largest value over the 64 lanes of a wavefront, every lane gets it.
__device__ __forceinline__ double wave_max(double v) {
  union { double d; int i[2]; } a, b;
  a.d = v;
  // xor 1, xor 2, half-row mirror, row mirror: the maximum of each row of 16
  b.i[0] = __builtin_amdgcn_update_dpp(0, a.i[0], 0xB1, 0xF, 0xF, false);
  b.i[1] = __builtin_amdgcn_update_dpp(0, a.i[1], 0xB1, 0xF, 0xF, false);
  a.d = fmax(a.d, b.d);
  b.i[0] = __builtin_amdgcn_update_dpp(0, a.i[0], 0x4E, 0xF, 0xF, false);
  b.i[1] = __builtin_amdgcn_update_dpp(0, a.i[1], 0x4E, 0xF, 0xF, false);
  a.d = fmax(a.d, b.d);
  b.i[0] = __builtin_amdgcn_update_dpp(0, a.i[0], 0x141, 0xF, 0xF, false);
  b.i[1] = __builtin_amdgcn_update_dpp(0, a.i[1], 0x141, 0xF, 0xF, false);
  a.d = fmax(a.d, b.d);
  b.i[0] = __builtin_amdgcn_update_dpp(0, a.i[0], 0x140, 0xF, 0xF, false);
  b.i[1] = __builtin_amdgcn_update_dpp(0, a.i[1], 0x140, 0xF, 0xF, false);
  a.d = fmax(a.d, b.d);
  a.d = fmax(a.d, __shfl_xor(a.d, 16, 64));
  a.d = fmax(a.d, __shfl_xor(a.d, 32, 64));
  return a.d;
}

// value of v in lane `lane` (wave-uniform)
__device__ __forceinline__ double lane_value(double v, int lane) {
  union { double d; int i[2]; } a;
  a.d = v;
  a.i[0] = __builtin_amdgcn_readlane(a.i[0], lane);
  a.i[1] = __builtin_amdgcn_readlane(a.i[1], lane);
  return a.d;
}

// Pivot key: the non-negative value with its lowest 6 mantissa bits replaced
// by 63 - index, so that the largest key picks the largest value (to 2^-46
// relative) and, among equal ones, the smallest index.  Read back as a
// double, keys of non-negative values keep their order.
__device__ __forceinline__ double pivot_key(double v, int i) {
  const double c = v > 0.0 ? v : 0.0;
  return __longlong_as_double((__double_as_longlong(c) & ~63ll) | (long long)(63 - i));
}

// Cholesky factorisation of the symmetric n x n matrix G (LDS, ld LDA; only
// the upper triangle is read), optionally with diagonal pivoting:
//   G[perm, perm] = R^T R,  R upper triangular (left in G, ld LDA),
// where perm = identity without pivoting; with pivoting, step k takes the
// largest remaining diagonal entry of the Schur complement (the column order
// of pivoted QR of the matrix whose Gram G is).  X (LDS, ld LDA) is scratch.
// A pivot not larger than 1e-20 times the column's own initial diagonal
// marks a numerically dependent column: the pivot is replaced by 1 so the
// factorisation continues as if the column were a fresh unit direction, and
// dep[k] is set (the caller replaces that column of Q by a pseudo-random
// vector and zeroes row k of R).  A non-finite pivot latches FLAG_NONFINITE
// and is treated the same way.
// The elimination runs in the original index space (pivoting only chooses
// the next index), each thread owning fixed upper-triangle entries; a step
// issues all its LDS reads at once and ends with the only barrier.  With
// pivoting every wavefront finds the pivot itself (maximum of packed
// value/index keys over its lanes).
template <int NO, bool PIVOT>
__device__ __forceinline__ void chol_piv(const Dev& d, double* G, double* X, int n, int* perm, int* dep) {
  __shared__ double diag0[CAP];
  __shared__ double dpiv[CAP];
  int oi[NO], oj[NO];
  owned_pairs<NO>(n, oi, oj);
  const int j = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  if (threadIdx.x < n) diag0[threadIdx.x] = G[threadIdx.x * (LDA + 1)];
  __syncthreads();
  uint64_t done = 0;  // indices already eliminated (identical in every thread)
  for (int k = 0; k < n; ++k) {
    int p = k;
    double dk;
    if (PIVOT) {
      const bool cand = lane < n && !((done >> lane) & 1);
      const double v = cand ? G[lane * (LDA + 1)] : 0.0;
      const double kmax = wave_max(cand ? pivot_key(v, lane) : 0.0);
      p = 63 - (int)(__double_as_longlong(kmax) & 63);
      dk = lane_value(v, p);
    } else {
      dk = G[k * (LDA + 1)];
    }
    const double d0 = diag0[p];
    // pivot row (Schur values at this step) in the original index space
    const double xrec = (threadIdx.x < n) ? G[(lane < p ? lane : p) + (lane < p ? p : lane) * LDA] : 0.0;
    double gpi[NO], gpj[NO], gij[NO];
    bool act[NO];
#pragma unroll
    for (int m = 0; m < NO; ++m) {
      const int i = oi[m], jj = oj[m];
      act[m] = PIVOT ? (i >= 0 && !((done >> i) & 1) && !((done >> jj) & 1) && i != p && jj != p) : (i > k);
      if (act[m]) {
        gpi[m] = G[(i < p ? i : p) + (i < p ? p : i) * LDA];
        gpj[m] = G[(jj < p ? jj : p) + (jj < p ? p : jj) * LDA];
        gij[m] = G[i + jj * LDA];
      }
    }
    bool isdep = false;
    if (!isfinite(dk)) {
      dk = 1.0;
      isdep = true;
      if (threadIdx.x == 0) atomicOr(d.flags, FLAG_NONFINITE);
    } else if (!(dk > 1e-20 * d0)) {
      dk = 1.0;
      isdep = true;
    }
    const double inv = rcp_nr(dk);
    done |= 1ull << p;
    if (threadIdx.x == 0) {
      perm[k] = p;
      dep[k] = isdep ? 1 : 0;
      dpiv[k] = dk;
    }
    if (threadIdx.x < n) X[k + threadIdx.x * LDA] = xrec;
#pragma unroll
    for (int m = 0; m < NO; ++m)
      if (act[m]) G[oi[m] + oj[m] * LDA] = fma(-gpi[m] * inv, gpj[m], gij[m]);
    __syncthreads();
  }
  if (threadIdx.x < n) dpiv[threadIdx.x] = sqrt(dpiv[threadIdx.x]);
  __syncthreads();
  // R[k][l] = (pivot row k at column perm[l]) / rdiag[k] for l > k
  if (j < n) {
    const int pl = perm[j];
    for (int k = g; k < n; k += 4) {
      double v = 0.0;
      if (j == k) v = dpiv[k];
      else if (j > k) v = X[k + pl * LDA] * rcp_nr(dpiv[k]);
      G[k + j * LDA] = v;
    }
  }
  __syncthreads();
}

// X = R^{-1} for upper triangular R (both LDS, ld LDA), right-looking back
// substitution with one barrier per step: once rows > k have been removed
// from row k, row k is final up to the factor 1/R[k][k] and is removed from
// all rows above in parallel (each thread owning fixed entries, reads first).
template <int NO>
__device__ __forceinline__ void tri_inv(const double* R, double* X, int n) {
  __shared__ double rinv[CAP];
  int oi[NO], oj[NO];
  owned_pairs<NO>(n, oi, oj);
  const int j = threadIdx.x & 63, g = threadIdx.x >> 6;
  if (j < n)
    for (int i = g; i < n; i += 4) X[i + j * LDA] = (i == j) ? 1.0 : 0.0;
  if (threadIdx.x < n) rinv[threadIdx.x] = 1.0 / R[threadIdx.x * (LDA + 1)];
  __syncthreads();
  for (int k = n - 1; k > 0; --k) {
    const double rk = rinv[k];
    double rik[NO], xkj[NO], xij[NO];
    bool act[NO];
#pragma unroll
    for (int m = 0; m < NO; ++m) {
      act[m] = oi[m] >= 0 && oi[m] < k && oj[m] >= k;
      if (act[m]) {
        rik[m] = R[oi[m] + k * LDA];
        xkj[m] = X[k + oj[m] * LDA];
        xij[m] = X[oi[m] + oj[m] * LDA];
      }
    }
#pragma unroll
    for (int m = 0; m < NO; ++m)
      if (act[m]) X[oi[m] + oj[m] * LDA] = fma(-rik[m] * rk, xkj[m], xij[m]);
    __syncthreads();
  }
  if (j < n)
    for (int i = g; i < n; i += 4) X[i + j * LDA] *= rinv[i];
  __syncthreads();
}

// smallest k with (sum_{j >= k} sig_j^2)^(1/2) <= tol (Algorithms 4, 5)
__device__ __forceinline__ int tail_rank(const double* sig, int n, double tol) {
  double tail2 = 0.0;
  int k = n;
  for (int j = n - 1; j >= 0; --j) {
    tail2 += sig[j] * sig[j];
    if (sqrt(tail2) <= tol) k = j;
    else break;
  }
  return k;
}

// dst (LDS, ld LDA) = src (rows x cols, ld lds), eight loads in flight per thread
__device__ __forceinline__ void copy_to_lds(double* dst, const double* src, int lds, int rows, int cols) {
  const int n = rows * cols;
  for (int base = threadIdx.x; base < n; base += 8 * NTHR) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * NTHR;
      v[u] = idx < n ? src[(idx % rows) + (idx / rows) * lds] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * NTHR;
      if (idx < n) dst[(idx % rows) + (idx / rows) * LDA] = v[u];
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void copy_from_lds(double* dst, int ldd, const double* src, int rows, int cols, double scale) {
  for (int idx = threadIdx.x; idx < rows * cols; idx += NTHR) {
    const int i = idx % rows, j = idx / rows;
    dst[i + j * ldd] = scale * src[i + j * LDA];
  }
  __syncthreads();
}

}  // namespace dd
