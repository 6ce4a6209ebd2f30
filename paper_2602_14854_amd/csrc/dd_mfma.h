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
