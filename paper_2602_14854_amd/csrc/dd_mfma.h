// FP64 matrix-core building blocks for the tall-skinny kernels (gfx950,
// v_mfma_f64_16x16x4f64).  D = A (16 x 4) * B (4 x 16) + C with
//   lane l supplies a = A[l % 16][l / 16] and b = B[l / 16][l % 16],
//   component v of lane l holds D[4 v + l / 16][l % 16].
//
// A wavefront works on strips of 16 rows.  The product of a strip X (16 x k)
// with a small matrix B (k x n) is formed as Y^T = B^T X^T: B^T comes from
// LDS as ready-made operand fragments, X^T straight from global memory (lane
// l reads row l % 16, column 4 ks + l / 16: 16 consecutive rows per column),
// and component v of the accumulator for column block cb holds
// Y[l % 16][16 cb + 4 v + l / 16], so its store writes 16 consecutive rows.
//
// Gram-type reductions (sum over rows of X[row][i] Y[row][j]) take both
// operands as fragments f[b] with lane l holding X[kk + l / 16][16 b + l % 16];
// a strip is first written row-major into a per-wavefront LDS buffer.
#pragma once

#include "dd_internal.h"

namespace dd {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int NW = NTHR / 64;   // wavefronts per workgroup

__device__ inline dbl4 mfma64(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline dbl4 zero4() {
  dbl4 z = {0.0, 0.0, 0.0, 0.0};
  return z;
}

template <int NA>
__device__ inline void zero_acc(dbl4* a) {
#pragma unroll
  for (int i = 0; i < NA; ++i) a[i] = zero4();
}

// ---------------------------------------------------------------------------
// Precision of the tall-skinny products.  P = 0: FP64 (v_mfma_f64_16x16x4f64);
// P = 1: FP32 operands, FP32 accumulation (v_mfma_f32_16x16x4f32); P = 2:
// split BF16, x = hi + lo with hi = bf16(x), lo = bf16(x - hi), and
// a b ~ hi_a hi_b + hi_a lo_b + lo_a hi_b accumulated in FP32
// (v_mfma_f32_16x16x32_bf16, three per product; its operand in lane l is
// A[l % 16][8 (l/16) + i], i < 8).  The FP32-accumulating instructions hold
// D[4 (l/16) + v][l % 16] in component v of lane l (the FP64 one
// D[4 v + l/16][l % 16]).
// Operands are handled in sub-steps u: lane (l16 = l % 16, kq = l / 16)
// holds column sub_col(u, kq) of its row.  For P = 0, 1 a sub-step is one
// 4-column instruction; for P = 2 eight consecutive sub-steps form one
// 32-column instruction whose lane operand is columns 32 g + 8 kq + 0..7.
// ---------------------------------------------------------------------------
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int P> struct Prec;
template <> struct Prec<0> { using F = double; using Acc = dbl4; };
template <> struct Prec<1> { using F = float; using Acc = flt4; };
template <> struct Prec<2> { using F = float; using Acc = flt4; };

template <int P>
__device__ __forceinline__ int sub_col(int u, int kq) {
  return P == 2 ? 32 * (u >> 3) + 8 * kq + (u & 7) : 4 * u + kq;
}

// column of the product held in component v of column block cb
template <int P>
__device__ __forceinline__ int out_col(int cb, int v, int kq) {
  return P == 0 ? 16 * cb + 4 * v + kq : 16 * cb + 4 * kq + v;
}

// lane group (l / 16) that holds product column c
template <int P>
__device__ __forceinline__ int out_kq(int c) {
  return P == 0 ? (c & 3) : ((c & 15) >> 2);
}

// sub-steps actually executed for k live columns (whole instructions)
template <int P>
__host__ __device__ constexpr int live_sub(int k) {
  return P == 2 ? 8 * ((k + 31) / 32) : (k + 3) / 4;
}

// sub-steps of an operand array covering a capacity of 16 nc columns
template <int P>
constexpr int sub_cap(int nc) {
  return P == 2 ? 8 * ((nc + 1) / 2) : 4 * nc;
}

template <int P>
__device__ __forceinline__ void zero_prod(typename Prec<P>::Acc* a, int n) {
  for (int i = 0; i < n; ++i) a[i] = typename Prec<P>::Acc{0, 0, 0, 0};
}

__device__ __forceinline__ void bf16_split(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

// acc[cb] += sum over the NSUB sub-steps u of (fragment u, block cb) x xv[u],
// cb < NCB.  frag[(u * NCL + cb) * 64 + lane] is the coefficient operand
// B[sub_col(u, kq)][16 cb + l16] (NCL column blocks per sub-step in the
// array, of which the first NCB are used); xv[u] the row's value in column
// sub_col(u, kq).  All NSUB sub-steps are issued (operands beyond the live
// columns are zero): a branch between matrix-core instructions would make
// the compiler copy the accumulators between register files around it.
template <int P, int NCB, int NSUB, int NCL = NCB>
__device__ __forceinline__ void prod_acc(typename Prec<P>::Acc* acc, const typename Prec<P>::F* frag,
                                         const typename Prec<P>::F* xv) {
  static_assert(NCB <= NCL, "column blocks beyond the fragment layout");
  const int lane = threadIdx.x & 63;
  if constexpr (P == 2) {
    static_assert(NSUB % 8 == 0, "split-BF16 operands come in whole 32-column instructions");
#pragma unroll
    for (int g = 0; g < NSUB / 8; ++g) {
      bf16x8 xh, xl;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        __bf16 h, l;
        bf16_split(xv[8 * g + i], h, l);
        xh[i] = h;
        xl[i] = l;
      }
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        bf16x8 ah, al;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          __bf16 h, l;
          bf16_split(frag[((8 * g + i) * NCL + cb) * 64 + lane], h, l);
          ah[i] = h;
          al[i] = l;
        }
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, xh, acc[cb], 0, 0, 0);
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, xl, acc[cb], 0, 0, 0);
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, xh, acc[cb], 0, 0, 0);
      }
    }
  } else {
#pragma unroll
    for (int u = 0; u < NSUB; ++u) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        if constexpr (P == 0)
          acc[cb] = mfma64(frag[(u * NCL + cb) * 64 + lane], xv[u], acc[cb]);
        else
          acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(frag[(u * NCL + cb) * 64 + lane], xv[u], acc[cb], 0, 0, 0);
      }
    }
  }
}

// doubles of LDS taken by n fragment values of precision P
template <int P>
constexpr size_t frag_doubles(size_t n) {
  return P == 0 ? n : (n + 1) / 2;
}

// leading dimension (doubles) of a row-major LDS strip with NCB column blocks
template <int NCB>
constexpr int strip_ld() { return 16 * NCB + 1; }

// Gram of a row-major LDS strip Ys (16 rows, leading dimension LD):
// g[blk(bi, bj)] += sum_rows Ys[row][16 bi + i] Ys[row][16 bj + j] for the
// upper block triangle bi <= bj, blocks ordered (0,0), (0,1), .., (1,1), ..
template <int NCB, int LD>
__device__ inline void strip_gram(dbl4* g, const double* Ys) {
  const int lane = threadIdx.x & 63;
  const int l16 = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 16; kk += 4) {
    double f[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) f[cb] = Ys[(kk + kq) * LD + 16 * cb + l16];
    int idx = 0;
#pragma unroll
    for (int bi = 0; bi < NCB; ++bi) {
#pragma unroll
      for (int bj = bi; bj < NCB; ++bj) {
        g[idx] = mfma64(f[bi], f[bj], g[idx]);
        ++idx;
      }
    }
  }
}

// Sum the wavefronts' accumulators over the workgroup in the fixed order
// ((w3 + w2) + w1) + w0; the total ends in wavefront 0.  red must hold
// NACC * 256 doubles of LDS that no wavefront still uses.  All threads call.
template <int NACC>
__device__ inline void wg_reduce_acc(dbl4* acc, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  for (int w = NW - 1; w >= 0; --w) {
    if (wave == w) {
#pragma unroll
      for (int a = 0; a < NACC; ++a) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double* p = red + (a * 4 + v) * 64 + lane;
          if (w == NW - 1) *p = acc[a][v];
          else if (w > 0) *p = *p + acc[a][v];
          else acc[a][v] = acc[a][v] + *p;
        }
      }
    }
    __syncthreads();
  }
}

// Workgroups whose wavefront pairs (0,1) and (2,3) accumulate different
// outputs: sum each pair in the order w_odd + w_even; the totals end in
// wavefronts 0 and 2.  red must hold 2 * NACC * 256 doubles of LDS that no
// wavefront still uses.  All threads call.
template <int NACC>
__device__ inline void pair_reduce_acc(dbl4* acc, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* r = red + (wave >> 1) * NACC * 256;
  __syncthreads();
  if (wave & 1) {
#pragma unroll
    for (int a = 0; a < NACC; ++a)
#pragma unroll
      for (int v = 0; v < 4; ++v) r[(a * 4 + v) * 64 + lane] = acc[a][v];
  }
  __syncthreads();
  if (!(wave & 1)) {
#pragma unroll
    for (int a = 0; a < NACC; ++a)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[a][v] = r[(a * 4 + v) * 64 + lane] + acc[a][v];
  }
}

// Store accumulator block (bi, bj) of a symmetric n x n matrix (leading
// dimension ld) and its mirror; in a diagonal block only i <= j writes, so
// every entry has one writer.
__device__ inline void store_sym_block(double* out, int ld, int n, int bi, int bj, dbl4 a, double scale) {
  const int lane = threadIdx.x & 63;
  const int l16 = lane & 15, kq = lane >> 4;
  const int j = 16 * bj + l16;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 16 * bi + 4 * v + kq;
    if (i < n && j < n && (bi != bj || i <= j)) {
      out[i + (int64_t)j * ld] = a[v] * scale;
      out[j + (int64_t)i * ld] = a[v] * scale;
    }
  }
}

// Store accumulator block (bi, bj) of a general na x nb matrix.
__device__ inline void store_block(double* out, int ld, int na, int nb, int bi, int bj, dbl4 a, double scale) {
  const int lane = threadIdx.x & 63;
  const int l16 = lane & 15, kq = lane >> 4;
  const int j = 16 * bj + l16;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 16 * bi + 4 * v + kq;
    if (i < na && j < nb) out[i + (int64_t)j * ld] = a[v] * scale;
  }
}

// Upper-block-triangle Gram accumulators (NB = NCB (NCB+1)/2) of wavefront 0
// to a symmetric n x n matrix with leading dimension n.
template <int NCB>
__device__ inline void store_gram(const dbl4* g, double* out, int n, double scale) {
  int idx = 0;
#pragma unroll
  for (int bi = 0; bi < NCB; ++bi) {
#pragma unroll
    for (int bj = bi; bj < NCB; ++bj) {
      store_sym_block(out, n, n, bi, bj, g[idx], scale);
      ++idx;
    }
  }
}

}  // namespace dd
