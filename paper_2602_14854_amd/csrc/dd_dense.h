// Dense FP64 building blocks for one workgroup (NTHR threads) working on
// small matrices in LDS: one-sided Jacobi SVD / eigensolver, Cholesky,
// triangular inverse, products, sorting and the tail rank rule.
#pragma once

#include <type_traits>

#include "dd_internal.h"
#include "dd_mfma.h"

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


// C (m x n) = alpha * op(A) op(B) + beta D for m, n, k <= CAP, where the
// addend D (ld ldd) is C itself (mm) or another buffer (mm_add); generic
// pointers (LDS or global), C aliasing neither A nor B.  On the FP64 matrix
// cores: the 16 x 16 output tiles are dealt to the wavefronts, and a
// wavefront issues every operand load of a tile (at clamped, always valid
// addresses; out-of-range values replaced by zero) before its first
// v_mfma_f64_16x16x4f64, so a tile costs one load latency instead of one
// per k.  The k loop has a compile-time length NK (steps of 4: k rounded up
// to 16, 32, 48 or 64) and runs as two accumulator chains.
template <int NK>
__device__ __forceinline__ void mm_body(double* C, int ldc, const double* A, int lda, bool ta, const double* B,
                                        int ldb, bool tb, int m, int n, int k, double alpha, double beta,
                                        const double* D, int ldd) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  const int tm = (m + 15) >> 4, tn = (n + 15) >> 4;
  // tile / tm for tile < 16 and tm <= 4 without a division
  const int magic = tm == 1 ? 64 : (tm == 2 ? 32 : (tm == 3 ? 22 : 16));
  for (int tile = wave; tile < tm * tn; tile += NW) {
    const int tj = (tile * magic) >> 6, ti = tile - tj * tm;
    const int i0 = 16 * ti, j0 = 16 * tj;
    const int i = i0 + l16, j = j0 + l16;  // A row and B column of this lane
    const int ic = i < m ? i : 0, jc = j < n ? j : 0;
    double av[NK], bv[NK];
#pragma unroll
    for (int s4 = 0; s4 < NK; ++s4) {
      const int l = 4 * s4 + kq;
      const int lc = l < k ? l : 0;
      av[s4] = ta ? A[lc + ic * lda] : A[ic + lc * lda];
      bv[s4] = tb ? B[jc + lc * ldb] : B[lc + jc * ldb];
    }
    dbl4 e = zero4(), o = zero4();
#pragma unroll
    for (int s4 = 0; s4 < NK; s4 += 2) {
      const int l = 4 * s4 + kq;
      e = mfma64((i < m && l < k) ? av[s4] : 0.0, (j < n && l < k) ? bv[s4] : 0.0, e);
      o = mfma64((i < m && l + 4 < k) ? av[s4 + 1] : 0.0, (j < n && l + 4 < k) ? bv[s4 + 1] : 0.0, o);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ci = i0 + 4 * v + kq, cj = j0 + l16;
      if (ci < m && cj < n) {
        const double acc = e[v] + o[v];
        const double dv = (beta == 0.0) ? 0.0 : beta * D[ci + (int64_t)cj * ldd];
        C[ci + (int64_t)cj * ldc] = (beta == 0.0) ? alpha * acc : fma(alpha, acc, dv);
      }
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void mm_add(double* C, int ldc, const double* A, int lda, bool ta, const double* B, int ldb,
                                       bool tb, int m, int n, int k, double alpha, double beta, const double* D,
                                       int ldd) {
  if (k <= 16) mm_body<4>(C, ldc, A, lda, ta, B, ldb, tb, m, n, k, alpha, beta, D, ldd);
  else if (k <= 32) mm_body<8>(C, ldc, A, lda, ta, B, ldb, tb, m, n, k, alpha, beta, D, ldd);
  else if (k <= 48) mm_body<12>(C, ldc, A, lda, ta, B, ldb, tb, m, n, k, alpha, beta, D, ldd);
  else mm_body<16>(C, ldc, A, lda, ta, B, ldb, tb, m, n, k, alpha, beta, D, ldd);
}

__device__ __forceinline__ void mm(double* C, int ldc, const double* A, int lda, bool ta, const double* B, int ldb,
                                   bool tb, int m, int n, int k, double alpha, double beta) {
  mm_add(C, ldc, A, lda, ta, B, ldb, tb, m, n, k, alpha, beta, C, ldc);
}

// One product C = alpha op(A) op(B) + beta D of mm_multi (same meaning and
// limits as the arguments of mm_add).
struct MMOp {
  double* C;
  int ldc;
  const double* A;
  int lda;
  bool ta;
  const double* B;
  int ldb;
  bool tb;
  int m, n, k;
  double alpha, beta;
  const double* D;
  int ldd;
};

// Several independent products in one pass: the 16 x 16 output tiles of
// all of them are dealt to the wavefronts together, so their operand loads
// overlap and the group costs one barrier instead of one per product (the
// tiles are formed exactly as by mm_add).  No product may read another's
// output.  All threads call.
template <int NK, int NP>
__device__ __forceinline__ void mm_multi_body(const MMOp (&ops)[NP]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  int first[NP + 1];
  first[0] = 0;
#pragma unroll
  for (int q = 0; q < NP; ++q) first[q + 1] = first[q] + ((ops[q].m + 15) >> 4) * ((ops[q].n + 15) >> 4);
  for (int tile = wave; tile < first[NP]; tile += NW) {
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      if (tile < first[q] || tile >= first[q + 1]) continue;
      const MMOp& o = ops[q];
      const int tm = (o.m + 15) >> 4;
      const int magic = tm == 1 ? 64 : (tm == 2 ? 32 : (tm == 3 ? 22 : 16));
      const int lt = tile - first[q];
      const int tj = (lt * magic) >> 6, ti = lt - tj * tm;
      const int i0 = 16 * ti, j0 = 16 * tj;
      const int i = i0 + l16, j = j0 + l16;
      const int ic = i < o.m ? i : 0, jc = j < o.n ? j : 0;
      double av[NK], bv[NK];
#pragma unroll
      for (int s4 = 0; s4 < NK; ++s4) {
        const int l = 4 * s4 + kq;
        const int lc = l < o.k ? l : 0;
        av[s4] = o.ta ? o.A[lc + ic * o.lda] : o.A[ic + lc * o.lda];
        bv[s4] = o.tb ? o.B[jc + lc * o.ldb] : o.B[lc + jc * o.ldb];
      }
      dbl4 e = zero4(), od = zero4();
#pragma unroll
      for (int s4 = 0; s4 < NK; s4 += 2) {
        const int l = 4 * s4 + kq;
        e = mfma64((i < o.m && l < o.k) ? av[s4] : 0.0, (j < o.n && l < o.k) ? bv[s4] : 0.0, e);
        od = mfma64((i < o.m && l + 4 < o.k) ? av[s4 + 1] : 0.0, (j < o.n && l + 4 < o.k) ? bv[s4 + 1] : 0.0, od);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ci = i0 + 4 * v + kq, cj = j0 + l16;
        if (ci < o.m && cj < o.n) {
          const double acc = e[v] + od[v];
          const double dv = (o.beta == 0.0) ? 0.0 : o.beta * o.D[ci + (int64_t)cj * o.ldd];
          o.C[ci + (int64_t)cj * o.ldc] = (o.beta == 0.0) ? o.alpha * acc : fma(o.alpha, acc, dv);
        }
      }
    }
  }
  __syncthreads();
}

template <int NP>
__device__ __forceinline__ void mm_multi(const MMOp (&ops)[NP]) {
  int k = 0;
#pragma unroll
  for (int q = 0; q < NP; ++q) k = ops[q].k > k ? ops[q].k : k;
  if (k <= 16) mm_multi_body<4, NP>(ops);
  else if (k <= 32) mm_multi_body<8, NP>(ops);
  else if (k <= 48) mm_multi_body<12, NP>(ops);
  else mm_multi_body<16, NP>(ops);
}

// C = alpha A B + beta D for zero-padded square LDS matrices of order 16 NT
// (ld LDA) whose result is symmetric (A and B symmetric and commuting, as
// for polynomials in one symmetric matrix), with B and D symmetric.  Only
// the tiles on and above the diagonal are formed, and each value is stored
// at (i, j) and (j, i), so C comes out exactly symmetric: iterations built
// on it keep exact symmetry, and B can be read along its columns
// (conflict-free).  C must differ from A, B and D unless beta is 0 (then D
// may be C).  Each tile runs two accumulator chains (even and odd k steps)
// to halve the dependent v_mfma_f64_16x16x4f64 sequence.  Entries past the
// order of the data are zero in A, B and D and stay zero in C.
template <int NT, int NK = 4 * NT>
__device__ __forceinline__ void sym_mm(double* C, const double* A, const double* B, double alpha, double beta,
                                       const double* D) {
  // NK k steps of 4 (even; 4 NK at least the order of the data, beyond which
  // the operands are zero)
  constexpr int NTILE = NT * (NT + 1) / 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  for (int tile = wave; tile < NTILE; tile += NW) {
    // tile -> (I, J), I <= J, column by column of the upper triangle
    int I = tile, J = 0;
#pragma unroll
    for (int c = 0; c < NT; ++c)
      if (I > J) {
        I -= J + 1;
        ++J;
      }
    const int i0 = 16 * I, j0 = 16 * J;
    double av[NK], bv[NK];
#pragma unroll
    for (int s4 = 0; s4 < NK; ++s4) {
      av[s4] = A[i0 + l16 + (4 * s4 + kq) * LDA];
      bv[s4] = B[j0 + l16 + (4 * s4 + kq) * LDA];
    }
    dbl4 e = zero4(), o = zero4();
#pragma unroll
    for (int s4 = 0; s4 < NK; s4 += 2) {
      e = mfma64(av[s4], bv[s4], e);
      o = mfma64(av[s4 + 1], bv[s4 + 1], o);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = i0 + 4 * v + kq, c = j0 + l16;
      const double acc = e[v] + o[v];
      const double val = beta == 0.0 ? alpha * acc : fma(alpha, acc, beta * D[r + c * LDA]);
      if (I < J || r <= c) {
        C[r + c * LDA] = val;
        C[c + r * LDA] = val;
      }
    }
  }
  __syncthreads();
}

// One block of a partial-sum reduction: dst (rows x cols, ldd) = scale *
// the sum over the workgroup partials of the block at offset off (leading
// dimension lds).
struct PartBlock {
  int off, lds, rows, cols;
  double* dst;
  int ldd;
  double scale;
};

// Sum up to NBLK blocks of ngp workgroup partials in one pass over the
// concatenated entries, in a fixed order over the partials (deterministic).
// Each thread takes E entries and U partials of each per round, E U = 32
// loads in flight, with U chosen from ngp so that few rounds remain;
// addresses of absent entries or partials are clamped to a valid one and the
// value dropped.  Blocks with rows * cols == 0 are skipped.  All threads call.
template <int NBLK>
__device__ __forceinline__ void sum_partials_blocks(const Dev& d, int s, int ngp, const PartBlock (&blk)[NBLK]) {
  const double* gp = gpart_of(d, s);
  int start[NBLK + 1];
  start[0] = 0;
#pragma unroll
  for (int b = 0; b < NBLK; ++b) start[b + 1] = start[b] + blk[b].rows * blk[b].cols;
  const int total = start[NBLK];
  auto run = [&](auto eu) {
    constexpr int E = decltype(eu)::value, U = 32 / E;
    for (int base = threadIdx.x; base < total; base += E * NTHR) {
      int src[E], bi[E], loc[E];
      double acc[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int idx = base + e * NTHR;
        bi[e] = -1;
        loc[e] = -1;
        src[e] = 0;
        // static block indices only (a runtime index into blk would put it
        // in scratch memory)
#pragma unroll
        for (int q = 0; q < NBLK; ++q) {
          if (idx >= start[q] && idx < start[q + 1]) {
            const int li = idx - start[q];
            bi[e] = q;
            loc[e] = li;
            src[e] = blk[q].off + (li % blk[q].rows) + (li / blk[q].rows) * blk[q].lds;
          }
        }
        acc[e] = 0.0;
      }
      for (int w0 = 0; w0 < ngp; w0 += U) {
        double v[E][U];
#pragma unroll
        for (int e = 0; e < E; ++e)
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int w = w0 + u < ngp ? w0 + u : 0;
            v[e][u] = gp[(int64_t)w * d.gpTile + src[e]];
          }
#pragma unroll
        for (int e = 0; e < E; ++e)
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (w0 + u < ngp) acc[e] += v[e][u];
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
#pragma unroll
        for (int q = 0; q < NBLK; ++q) {
          if (bi[e] == q)
            blk[q].dst[(loc[e] % blk[q].rows) + (loc[e] / blk[q].rows) * blk[q].ldd] = blk[q].scale * acc[e];
        }
      }
    }
  };
  using std::integral_constant;
  if (ngp > 8) run(integral_constant<int, 2>{});
  else if (ngp > 4) run(integral_constant<int, 4>{});
  else run(integral_constant<int, 8>{});
  __syncthreads();
}

// dst (rows x cols, ldd) = scale * sum over ngp workgroup partials of the
// block at offset off (leading dimension lds).
__device__ __forceinline__ void sum_partials(const Dev& d, int s, int ngp, int off, int lds, int rows, int cols, double* dst,
                             int ldd, double scale) {
  const PartBlock blk[1] = {{off, lds, rows, cols, dst, ldd, scale}};
  sum_partials_blocks<1>(d, s, ngp, blk);
}

// a double moved across lanes by the DPP pattern CTRL (every lane has a
// source in the patterns used here, so no old value is needed)
template <int CTRL>
__device__ __forceinline__ double dpp_double(double v) {
  union { double d; int i[2]; } a, b;
  a.d = v;
  b.i[0] = __builtin_amdgcn_mov_dpp(a.i[0], CTRL, 0xF, 0xF, true);
  b.i[1] = __builtin_amdgcn_mov_dpp(a.i[1], CTRL, 0xF, 0xF, true);
  return b.d;
}

// sum over aligned groups of G lanes (G = 1, 2, 4, 8 or 16) with DPP; each
// step adds a lane's partner, so every lane of a group ends with the same
// bits
template <int G>
__device__ __forceinline__ double group_sum_dpp(double v) {
  if (G == 1) return v;
  v += dpp_double<0xB1>(v);   // quad_perm [1,0,3,2]: partner lane ^ 1
  if (G == 2) return v;
  v += dpp_double<0x4E>(v);   // quad_perm [2,3,0,1]: partner lane ^ 2
  if (G == 4) return v;
  v += dpp_double<0x141>(v);  // row_half_mirror: lane i <-> 7 - i in each 8 (quads are uniform)
  if (G == 8) return v;
  v += dpp_double<0x140>(v);  // row_mirror: lane i <-> 15 - i in each row of 16
  return v;
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

// True when a further Jacobi sweep over B (rows x n, LDS, ld LDA) would not
// rotate any pair: no |b_p . b_q| exceeds tol ||b_p|| ||b_q|| among columns
// above the noise floor.  All the inner products at once on the FP64 matrix
// cores (the tiles of B^T B on and above the diagonal into Gq, LDS, ld LDA;
// NK = rows/4 rounded up), instead of the n - 1 rounds of a sweep.  flag is
// LDS scratch.
template <int NK>
__device__ __forceinline__ bool jacobi_quiet(const double* B, int rows, int n, double tol2, double floor2, double* Gq,
                                             int* flag) {
  if (threadIdx.x == 0) *flag = 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  const int tn = (n + 15) >> 4;
  for (int tile = wave; tile < tn * (tn + 1) / 2; tile += NW) {
    int I = tile, J = 0;
#pragma unroll
    for (int c = 0; c < CAP / 16; ++c)
      if (I > J) {
        I -= J + 1;
        ++J;
      }
    const int i = 16 * I + l16, j = 16 * J + l16;  // columns p (A side) and q (B side) of this lane
    const int ic = i < n ? i : 0, jc = j < n ? j : 0;
    double av[NK], bv[NK];
#pragma unroll
    for (int s4 = 0; s4 < NK; ++s4) {
      const int l = 4 * s4 + kq;
      const int lc = l < rows ? l : 0;
      av[s4] = B[lc + ic * LDA];
      bv[s4] = B[lc + jc * LDA];
    }
    dbl4 e = zero4(), o = zero4();
#pragma unroll
    for (int s4 = 0; s4 < NK; s4 += 2) {
      const int l = 4 * s4 + kq;
      e = mfma64((i < n && l < rows) ? av[s4] : 0.0, (j < n && l < rows) ? bv[s4] : 0.0, e);
      o = mfma64((i < n && l + 4 < rows) ? av[s4 + 1] : 0.0, (j < n && l + 4 < rows) ? bv[s4 + 1] : 0.0, o);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int p = 16 * I + 4 * v + kq, q = 16 * J + l16;
      if (p <= q && q < n) Gq[p + q * LDA] = e[v] + o[v];
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * n; idx += NTHR) {
    const int p = idx % n, q = idx / n;
    if (p < q) {
      const double ga = Gq[p + q * LDA], al = Gq[p * (LDA + 1)], be = Gq[q * (LDA + 1)];
      if (ga != 0.0 && al > floor2 && be > floor2 && ga * ga > tol2 * al * be) *flag = 1;
    }
  }
  __syncthreads();
  return *flag == 0;
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
// From the second sweep on, a sweep that rotated something is followed by
// the all-pairs test of jacobi_quiet: when it passes, the next sweep would
// only confirm convergence, and is skipped.
// Returns the number of sweeps (negative if not converged).
template <int G, int RPL, bool ACCV>
__device__ __forceinline__ int jacobi_1s_g(const Dev& d, double* B, int rows, int n, double* V, double tol, double floor_rel,
                           int max_sweeps, double* Gq) {
  __shared__ int rotated[3];  // per-sweep flags: set, read, cleared in rotation
  __shared__ double red[NTHR];
  __shared__ int bigrot[3];   // per-sweep flags of rotations with |sin| > 1e-6
  __shared__ int qflag;
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
  if (threadIdx.x < 3) bigrot[threadIdx.x] = 0;
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
    if (threadIdx.x == 0) bigrot[(sweep + 1) % 3] = 0;
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
        if (lane == 0 && fabs(sn) > 1e-6) bigrot[slot] = 1;
      }
      if (++va >= nm1) va -= nm1;
      if (++vb >= nm1) vb -= nm1;
      __syncthreads();
    }
    if (!rotated[slot]) {
      converged = true;
      break;
    }
    // a sweep that would rotate nothing only confirms convergence: after a
    // sweep of small rotations only, test all pairs at once instead
    if (sweep >= 1 && !bigrot[slot] && jacobi_quiet<(G * RPL + 3) / 4>(B, rows, n, tol2, floor2, Gq, &qflag)) {
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
  __shared__ double Gq[LDA * CAP];  // all-pairs test scratch
  if (n <= 32 && rows <= 32) {
    if (V) return jacobi_1s_g<16, 2, true>(d, B, rows, n, V, tol, floor_rel, max_sweeps, Gq);
    return jacobi_1s_g<16, 2, false>(d, B, rows, n, V, tol, floor_rel, max_sweeps, Gq);
  }
  if (V) return jacobi_1s_g<8, 8, true>(d, B, rows, n, V, tol, floor_rel, max_sweeps, Gq);
  return jacobi_1s_g<8, 8, false>(d, B, rows, n, V, tol, floor_rel, max_sweeps, Gq);
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

// X = R^{-1} for an upper triangular R (n x n in LDS, ld LDA, n <= 16 NT),
// by 16 x 16 blocks: the padding of R up to order 16 ceil(n/16) is set to
// the identity, wavefront I inverts the diagonal block R_II by back
// substitution (lane q < 16 holds column q; the rows of R_II are broadcast
// LDS reads), and the off-diagonal blocks follow by superdiagonals,
//   X_IJ = -X_II (sum_{K=I+1..J} R_IK X_KJ),
// one wavefront per block, on the FP64 matrix cores: the inner sum leaves
// the MFMA accumulator in exactly the layout of the B operand of the outer
// product, so it never goes through LDS.  X comes out zero below the
// diagonal and identity in the padding.
template <int NT>
__device__ __forceinline__ void tri_inv_blocked(double* R, double* X, int n) {
  __shared__ double dinv[16 * NT];
  const int nb = (n + 15) >> 4, np = 16 * nb;
  for (int idx = threadIdx.x; idx < np * np; idx += NTHR) {
    const int i = idx % np, j = idx / np;
    if (i >= n || j >= n) R[i + j * LDA] = i == j ? 1.0 : 0.0;
    if (i > j || (i >> 4) != (j >> 4)) X[i + j * LDA] = 0.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < np; i += NTHR) dinv[i] = rcp_nr(R[i * (LDA + 1)]);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (wave < nb && lane < 16) {
    const int b0 = 16 * wave, q = lane;
    double x[16];
#pragma unroll
    for (int i = 15; i >= 0; --i) {
      double acc = i == q ? 1.0 : 0.0;
#pragma unroll
      for (int l = i + 1; l < 16; ++l) acc = fma(-R[b0 + i + (b0 + l) * LDA], x[l], acc);
      x[i] = acc * dinv[b0 + i];
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) X[b0 + i + (b0 + q) * LDA] = i <= q ? x[i] : 0.0;
  }
  __syncthreads();
  const int l16 = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int dd = 1; dd < NT; ++dd) {
    if (dd < nb) {
      const int I = wave, J = wave + dd;
      if (J < nb) {
        const int i0 = 16 * I, j0 = 16 * J;
        dbl4 e = zero4(), o = zero4();
#pragma unroll
        for (int K = 1; K <= dd; ++K) {
          const int k0 = 16 * (I + K);
#pragma unroll
          for (int s4 = 0; s4 < 4; s4 += 2) {
            e = mfma64(R[i0 + l16 + (k0 + 4 * s4 + kq) * LDA], X[k0 + 4 * s4 + kq + (j0 + l16) * LDA], e);
            o = mfma64(R[i0 + l16 + (k0 + 4 * s4 + 4 + kq) * LDA], X[k0 + 4 * s4 + 4 + kq + (j0 + l16) * LDA], o);
          }
        }
        const dbl4 t = e + o;  // T = sum_K R_IK X_KJ, row 4v + kq, column l16
        dbl4 y = zero4();
#pragma unroll
        for (int v = 0; v < 4; ++v) y = mfma64(X[i0 + l16 + (i0 + 4 * v + kq) * LDA], t[v], y);
#pragma unroll
        for (int v = 0; v < 4; ++v) X[i0 + 4 * v + kq + (j0 + l16) * LDA] = -y[v];
      }
      __syncthreads();
    }
  }
}


// Cholesky factorisation of the symmetric n x n matrix G (n <= NMAX; LDS, ld
// LDA, upper triangle read), optionally with diagonal pivoting,
//   G[perm, perm] = R^T R,  R upper triangular,
// and the inverse R^{-1}.  The factor is formed by wavefront 0 alone with no
// workgroup barrier: lane j keeps row entries R[0..k][j] of its own (original) column
// j in registers and its current Schur diagonal.  Step k (left-looking):
// the pivot p is k, or with pivoting the largest remaining Schur diagonal
// (smallest index among equal ones); every lane forms
//   R[k][j] = (G[p][j] - sum_{l<k} R[l][p] R[l][j]) / R[k][p],
// reading R[l][p] from the LDS buffer Rt (CAP x (CAP + 1) doubles), where
// lane p stored row entry R[k][p] when it formed it: broadcast reads, no
// v_readlane chain.  A pivot not larger than 1e-20
// times the column's own initial diagonal (or non-finite) marks a
// numerically dependent column: the pivot is replaced by 1 (the Schur row is
// kept as the row of R) and dep[k] is set; the caller completes Q with a
// pseudo-random column there and zeroes row k of R.  The inverse follows by
// 16 x 16 blocks on all wavefronts (tri_inv_blocked).  On return (after a
// barrier): G = R (pivot order: column k of R belongs to original column
// perm[k]; upper, zero below, identity padding to a multiple of 16), X =
// R^{-1} (same layout), perm, dep.  All threads call.
template <int NMAX, bool PIVOT>
__device__ __forceinline__ void chol_inv_wave(const Dev& d, double* G, double* X, int n, int* perm, int* dep,
                                              double* Rt) {
  if (threadIdx.x < 64) {
    const int j = threadIdx.x;
    double rc[NMAX];  // rc[l] = R[l][j]
    double dg = j < n ? G[j * (LDA + 1)] : 0.0;
    const double d0 = dg;
    bool done = j >= n;
    int myk = -1;
    int pk[NMAX];  // pivot index of each step (wave-uniform)
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
      rc[k] = 0.0;
      pk[k] = k;
      if (k < n) {
        int p = k;
        if (PIVOT) {
          const double kmax = wave_max(done ? 0.0 : pivot_key(dg, j));
          p = 63 - (int)(__double_as_longlong(kmax) & 63);
        }
        pk[k] = p;
        const double g = G[(p < j ? p : j) + (p < j ? j : p) * LDA];
        double dk = lane_value(dg, p);
        const double d0k = lane_value(d0, p);
        bool isdep = false;
        if (!isfinite(dk)) {
          dk = 1.0;
          isdep = true;
          if (j == 0) atomicOr(d.flags, FLAG_NONFINITE);
        } else if (!(dk > 1e-20 * d0k)) {
          dk = 1.0;
          isdep = true;
        }
        const double rinv = rsqrt_nr(dk);
        // R[l][p], l < k: the pivot lane's entries, written to Rt at the
        // steps that formed them; broadcast reads (one address per wave)
        const double* rp = Rt + p * (CAP + 1);
        double a0 = g, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
        for (int l = 0; l < k; l += 4) {
          a0 = fma(-rp[l], rc[l], a0);
          if (l + 1 < k) a1 = fma(-rp[l + 1], rc[l + 1], a1);
          if (l + 2 < k) a2 = fma(-rp[l + 2], rc[l + 2], a2);
          if (l + 3 < k) a3 = fma(-rp[l + 3], rc[l + 3], a3);
        }
        const double rkj = (a0 + a1) + (a2 + a3);
        if (j == p) {
          rc[k] = dk * rinv;
          done = true;
          myk = k;
        } else if (!done) {
          rc[k] = rkj * rinv;
          dg = fma(-rc[k], rc[k], dg);
          Rt[j * (CAP + 1) + k] = rc[k];
        }
        if (j == 0) {
          perm[k] = p;
          dep[k] = isdep ? 1 : 0;
        }
      }
    }
    // R P: the column of lane j is column myk of the permuted factor
    if (myk >= 0) {
#pragma unroll
      for (int i = 0; i < NMAX; ++i)
        if (i < n) G[i + myk * LDA] = i <= myk ? rc[i] : 0.0;
    }
  }
  __syncthreads();
  // X = R^{-1} (R upper triangular in G, pivot order), blockwise
  tri_inv_blocked<(NMAX + 15) / 16>(G, X, n);
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
