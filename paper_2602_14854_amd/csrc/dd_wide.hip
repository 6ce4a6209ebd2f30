// Kernels of the wide plan: the DD-DLRA step for capacities beyond the
// narrow kernels' register and LDS layouts -- stored ranks up to 64,
// intermediate ranks up to 128 and augmentation widths up to 192 (the
// adaptive configurations of Algorithms 4-5 whose ranks grow near sources).
//
// Tall-skinny products (Y = X B) hold the coefficient fragments of one chunk
// of output columns in LDS; the chunk index is blockIdx.z, so a product of n
// columns runs as ceil(n / chunk) column slices over the same rows, and the
// k dimension (up to 192) is walked in groups of 64 columns whose operand
// loads are issued one group ahead of the matrix-core instructions.  Gram and
// Galerkin reductions are separate launches (kw_xgram) that load both
// operands straight into the matrix-core lane layout and leave one 64 x 64
// block of one partial per workgroup.
//
// Small per-subdomain kernels run one workgroup per subdomain (1024
// threads; the two SVD kernels 512).  Matrices of order up to 128 sit in
// LDS; the augmentation Gram (order up to 192) is kept as a packed lower
// triangle.  The one-sided Jacobi SVD keeps its columns in registers: each
// lane group of 16 holds a few column pairs of a round-robin (caterpillar)
// ordering, a pair's rows spread over the group's lanes, so a wavefront works
// on four pairs at once; after each round only the columns at the ends of a
// group's run move, to the neighbouring group.
#include <algorithm>
#include <type_traits>

#include "dd_dlra.h"
#include "dd_dense.h"
#include "dd_wide.h"

namespace dd {

constexpr int WTHR = 512;          // threads of a wide tall-skinny product
constexpr int WNW = WTHR / 64;
constexpr int XTHR = 256;          // threads of a wide reduction (kw_xgram)
constexpr int STHR = 1024;         // threads of a wide small kernel
constexpr int SNW = STHR / 64;
constexpr int WLD = WCAP_T + 1;    // leading dimension of LDS matrices of order <= 128
template <int V>
using wint = std::integral_constant<int, V>;

__host__ __device__ constexpr int wdiv(int a, int b) { return (a + b - 1) / b; }

// ============================================================================
// tall-skinny products
// ============================================================================

// Fragments of output columns [c0, c0 + 16 NCB) of B (k x n, ld bld) for ng
// groups of 64 rows of B: frag[((g 16 + u) NCB + cb) 64 + lane] =
// B[64 g + sub_col(u, lane / 16)][c0 + 16 cb + lane % 16].
template <int P, int NCB>
__device__ __forceinline__ void stage_frags(typename Prec<P>::F* frag, const double* B, int bld, int k, int n, int c0,
                                            int ng) {
  using F = typename Prec<P>::F;
  const int total = ng * 16 * NCB * 64;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int l = idx & 63, f = idx >> 6, cb = f % NCB, u = f / NCB;
    const int kc = 64 * (u >> 4) + sub_col<P>(u & 15, l >> 4), col = c0 + 16 * cb + (l & 15);
    frag[idx] = (kc < k && col < n) ? (F)B[kc + (int64_t)col * bld] : (F)0;
  }
}

// Y[:, c0 + j] = diag(rowscale) X B[:, c0 + j], c0 = 16 NCB blockIdx.z; X
// rows x k (ld rows), B k x n in the small workspace.  Columns flagged in the
// fill mask get deterministic pseudo-random values; with set_rank, one
// workgroup of each subdomain commits the truncated rank.
template <class SI, class SO, int P, int NCB>
__global__ __launch_bounds__(WTHR, P == 2 ? 2 : 4)  // four wavefronts per SIMD (two for split BF16)
void kw_gemm(Dev d, int axis, int sd0, const void* X, int64_t xsd, int rows, int kdim, int ndim, int boff, int bld,
             void* Y, int64_t ysd, const double* rowscale, int fill_off, int set_rank, int skip_off) {
  using F = typename Prec<P>::F;
  using Acc = typename Prec<P>::Acc;
  const int s = sd0 + blockIdx.y;
  const int k = dim_of(d, s, axis, kdim);
  const int n = dim_of(d, s, axis, ndim);
  const int c0 = blockIdx.z * 16 * NCB;
  if (set_rank && blockIdx.x == 0 && blockIdx.z == 0 && threadIdx.x == 0) d.rank[s] = d.rnew[s];
  if (c0 >= n || k <= 0) return;
  if (skip_off >= 0 && small_of(d, s)[skip_off] != 0.0) {
    // a skipped Cholesky-QR pass (B = I): Y = X on this block of columns
    const SI* Xc = (const SI*)X + (int64_t)s * xsd;
    SO* Yc = (SO*)Y + (int64_t)s * ysd;
    const int64_t tot = (int64_t)min(16 * NCB, n - c0) * rows;
    for (int64_t idx = (int64_t)blockIdx.x * WTHR + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * WTHR) {
      const int64_t o = (int64_t)c0 * rows + idx;
      Yc[o] = (SO)Xc[o];
    }
    return;
  }
  const int ng = wdiv(k, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  extern __shared__ double lds[];
  F* frag = reinterpret_cast<F*>(lds);
  __shared__ int fillm[16 * NCB];
  const double* sm = small_of(d, s);
  stage_frags<P, NCB>(frag, sm + boff, bld, k, n, c0, ng);
  for (int j = threadIdx.x; j < 16 * NCB; j += WTHR)
    fillm[j] = (fill_off >= 0 && c0 + j < n) ? (sm[fill_off + c0 + j] != 0.0) : 0;
  __syncthreads();
  const SI* Xs = (const SI*)X + (int64_t)s * xsd;
  SO* Ys = (SO*)Y + (int64_t)s * ysd;
  const int nst = wdiv(rows, 16);
  const int stride = gridDim.x * WNW;
  // NS sub-steps of each 64-column group of X and NC column blocks of the
  // output are issued; a subdomain of low rank (one group with few live
  // columns, few output columns) takes a shorter instance
  auto run = [&](auto ns_c, auto nc_c) {
    constexpr int NS = decltype(ns_c)::value, NC = decltype(nc_c)::value;
    // a group's NS sub-steps go in chunks of SUB (one instruction's worth:
    // 4 sub-steps, or 8 for the split-BF16 32-column instruction), the next
    // chunk's operands loaded while the current one's MFMAs run; so few
    // values in flight per lane keep the kernel at four wavefronts per SIMD
    constexpr int SUBI = P == 2 ? 8 : 4;
    constexpr int SUB = NS < SUBI ? NS : SUBI, NH = NS / SUB;
    F xv[SUB], xn[SUB];
    auto load = [&](int st_, int g_, int h_) {
      const int row_ = st_ * 16 + l16;
      const int rc = row_ < rows ? row_ : rows - 1;
#pragma unroll
      for (int u = 0; u < SUB; ++u) {
        const int kc = 64 * g_ + sub_col<P>(SUB * h_ + u, kq);
        const bool in = row_ < rows && kc < k;
        const SI v = Xs[(unsigned)((in ? kc : 0) * rows + rc)];  // offsets within a slab fit in 32 bits
        xn[u] = in ? (F)v : (F)0;
      }
    };
    int st = blockIdx.x * WNW + wave, g = 0, h = 0;
    if (st < nst) load(st, 0, 0);
    Acc acc[NC];
    zero_prod<P>(acc, NC);
    while (st < nst) {
#pragma unroll
      for (int u = 0; u < SUB; ++u) xv[u] = xn[u];
      int st2 = st, g2 = g, h2 = h + 1;
      if (h2 >= NH) {
        h2 = 0;
        g2 = g + 1;
        if (g2 >= ng) {
          g2 = 0;
          st2 = st + stride;
        }
      }
      if (st2 < nst) load(st2, g2, h2);
      prod_acc<P, NC, SUB, NCB>(acc, frag + (g * 16 + SUB * h) * NCB * 64, xv);
      if (g == ng - 1 && h == NH - 1) {
        const int row = st * 16 + l16;
        const bool rin = row < rows;
        const double rs = (rowscale != nullptr && rin) ? rowscale[row] : 1.0;
#pragma unroll
        for (int cb = 0; cb < NC; ++cb) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int j = out_col<P>(cb, v, kq);
            double val = (double)acc[cb][v] * rs;
            if (fillm[j]) val = hash_unit(((uint64_t)s << 40) ^ ((uint64_t)(c0 + j) << 24) ^ (uint64_t)row);
            if (rin && c0 + j < n) Ys[(int64_t)(c0 + j) * rows + row] = (SO)val;
          }
        }
        zero_prod<P>(acc, NC);
      }
      st = st2;
      g = g2;
      h = h2;
    }
  };
  constexpr int NS1 = P == 2 ? 8 : 4;  // one matrix-core instruction (P = 2: one 32-column one)
  const int ls = live_sub<P>(k), nl = n - c0;
  if (ng == 1 && ls <= NS1 && nl <= 16) run(wint<NS1>{}, wint<1>{});
  else if (ng == 1 && ls <= 8 && nl <= 32 && NCB >= 2) run(wint<8>{}, wint<(NCB >= 2 ? 2 : 1)>{});
  else run(wint<16>{}, wint<NCB>{});
}

// Augmentation matrix (Algorithm 4, step 1), one source block per blockIdx.z
// (0: the subdomain, 1: its low neighbour, 2: its high neighbour):
//   A[q, off_b + j] = sqrt(w_q) (V_b S_b^T)[q, j],  j < r_b.
__global__ __launch_bounds__(WTHR) void kw_aug_form(Dev d, int axis, int sd0) {
  constexpr int NCB = 4;
  const int s = sd0 + blockIdx.y;
  const int b = blockIdx.z;
  const int lo = neighbour(d, s, axis, -1), hi = neighbour(d, s, axis, +1);
  const int nb = b == 0 ? s : (b == 1 ? lo : hi);
  if (nb < 0) return;
  const int rs = d.rank[s], rl = lo >= 0 ? d.rank[lo] : 0;
  const int off = b == 0 ? 0 : (b == 1 ? rs : rs + rl);
  const int rb = d.rank[nb];
  const int M = d.M, R = d.R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  extern __shared__ double lds[];
  double* frag = lds;  // 16 x NCB x 64
  const double* Sn = d.S + (int64_t)nb * R * R;
  for (int idx = threadIdx.x; idx < 16 * NCB * 64; idx += WTHR) {
    const int l = idx & 63, f = idx >> 6, cb = f % NCB, u = f / NCB;
    const int kc = sub_col<0>(u, l >> 4), col = 16 * cb + (l & 15);
    frag[idx] = (kc < rb && col < rb) ? Sn[col + (int64_t)kc * R] : 0.0;  // S^T
  }
  __syncthreads();
  const double* Vn = d.V + (int64_t)nb * M * R;
  double* As = d.A + (int64_t)s * M * d.MA + (int64_t)off * M;
  const int nst = wdiv(M, 16);
  const int stride = gridDim.x * WNW;
  // a source block of rank <= 16 takes the short instance (one column
  // block, four sub-steps)
  auto run = [&](auto ns_c, auto nc_c) {
    constexpr int NS = decltype(ns_c)::value, NC = decltype(nc_c)::value;
    for (int st = blockIdx.x * WNW + wave; st < nst; st += stride) {
      const int q = st * 16 + l16;
      const bool rin = q < M;
      const int qc = rin ? q : M - 1;
      double xv[NS];
#pragma unroll
      for (int u = 0; u < NS; ++u) {
        const int kc = sub_col<0>(u, kq);
        const bool in = rin && kc < rb;
        const double v = Vn[(int64_t)(in ? kc : 0) * M + qc];
        xv[u] = in ? v : 0.0;
      }
      dbl4 acc[NC];
      zero_acc<NC>(acc);
      prod_acc<0, NC, NS, NCB>(acc, frag, xv);
      const double swq = d.sw[qc];
#pragma unroll
      for (int cb = 0; cb < NC; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = out_col<0>(cb, v, kq);
          if (rin && j < rb) As[(int64_t)j * M + q] = acc[cb][v] * swq;
        }
    }
  };
  if (rb <= 16) run(wint<4>{}, wint<1>{});
  else run(wint<16>{}, wint<NCB>{});
}

// K-step of an advection stage (eq. advx_evolK / advy_evolK, Appendix A),
// fused with K = U (S T) and the inflow ghosts, for output columns
// [c0, c0 + 32), c0 = 32 blockIdx.z:
//   K1[p] = U[p] M0 + U[p-e] Mm + U[p+e] Mp,
// the missing row at the low face replaced by U[p] GLo + U_lo[its high face]
// GLoN and at the high face by U[p] GHi + U_hi[its low face] GHiN.  The
// stored-rank dimension (up to 64) is walked in groups of 32 columns, only
// as many as the ranks need.
template <class S, int P>
__global__ __launch_bounds__(WTHR) void kw_kstep(Dev d, int axis, int sd0) {
  using F = typename Prec<P>::F;
  using Acc = typename Prec<P>::Acc;
  constexpr int NCB = 2, KSP = 16, KG = 8;  // KG sub-steps = 32 columns per group
  const int s = sd0 + blockIdx.y;
  const int t = d.tdim[s];
  const int c0 = blockIdx.z * 16 * NCB;
  if (c0 >= t) return;
  const int lo = neighbour(d, s, axis, -1), hi = neighbour(d, s, axis, +1);
  const int r = d.rank[s], rl = lo >= 0 ? d.rank[lo] : 0, rh = hi >= 0 ? d.rank[hi] : 0;
  const int N = d.N, R = d.R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  extern __shared__ double lds[];
  constexpr int nfrag = 7 * KSP * NCB * 64;
  constexpr int bstride = KSP * NCB * 64;
  constexpr int gstride = KG * NCB * 64;
  F* Cf = reinterpret_cast<F*>(lds);
  {
    const double* sm = small_of(d, s);
    const int offs[7] = {d.oM0, d.oMm, d.oMp, d.oGLo, d.oGHi, d.oGLoN, d.oGHiN};
    const int rows[7] = {r, r, r, r, r, rl, rh};
    for (int idx = threadIdx.x; idx < nfrag; idx += WTHR) {
      const int l = idx & 63, f = idx >> 6, cb = f % NCB, u = (f / NCB) % KSP, m = f / (NCB * KSP);
      const int kc = 32 * (u / KG) + sub_col<P>(u % KG, l >> 4), col = c0 + 16 * cb + (l & 15);
      Cf[idx] = (kc < rows[m] && col < t) ? (F)sm[offs[m] + kc + col * R] : (F)0;
    }
  }
  __syncthreads();
  const int kgr = (r + 31) / 32, kgl = (rl + 31) / 32, kgh = (rh + 31) / 32;
  const double* Ub = d.U;
  const double* Us = Ub + (int64_t)s * N * R;
  const double* Ul = lo >= 0 ? Ub + (int64_t)lo * N * R : Ub;
  const double* Uh = hi >= 0 ? Ub + (int64_t)hi * N * R : Ub;
  S* K1 = (S*)d.K1 + (int64_t)s * N * d.T;
  const int e = axis == 0 ? 1 : d.lnx;
  const int na = axis == 0 ? d.lnx : d.lny;
  const int nst = wdiv(N, 16);
  const int stride = gridDim.x * WNW;
  // KGR sub-steps of each 32-column group and NC output column blocks are
  // issued: a subdomain whose own and neighbouring ranks fit one short group
  // and whose block has at most 16 live columns takes the short instance
  auto run = [&](auto kg_c, auto nc_c) {
    constexpr int KGR = decltype(kg_c)::value, NC = decltype(nc_c)::value;
    for (int st = blockIdx.x * WNW + wave; st < nst; st += stride) {
      const int p = st * 16 + l16;
      const bool rin = p < N;
      const int pc = rin ? p : N - 1;
      const int ia = axis == 0 ? pc % d.lnx : pc / d.lnx;
      const int f = axis == 0 ? pc / d.lnx : pc % d.lnx;
      const bool hm = rin && ia > 0, hp = rin && ia < na - 1;
      const bool flo = rin && ia == 0, fhi = rin && ia == na - 1;
      const int pm = hm ? pc - e : pc, pp = hp ? pc + e : pc;
      Acc acc[NC];
      zero_prod<P>(acc, NC);
      for (int kg = 0; kg < kgr; ++kg) {
        F u0[KGR], um[KGR], up[KGR];
#pragma unroll
        for (int u = 0; u < KGR; ++u) {
          const int kc = 32 * kg + sub_col<P>(u, kq);
          const bool kin = kc < r;
          const int64_t col = (int64_t)(kin ? kc : 0) * N;
          const double v0 = Us[col + pc], vm = Us[col + pm], vp = Us[col + pp];
          u0[u] = (rin && kin) ? (F)v0 : (F)0;
          um[u] = (hm && kin) ? (F)vm : (F)0;
          up[u] = (hp && kin) ? (F)vp : (F)0;
        }
        prod_acc<P, NC, KGR, NCB>(acc, Cf + kg * gstride, u0);
        prod_acc<P, NC, KGR, NCB>(acc, Cf + bstride + kg * gstride, um);
        prod_acc<P, NC, KGR, NCB>(acc, Cf + 2 * bstride + kg * gstride, up);
        // own face row: U[p] GLo at the low face, U[p] GHi at the high face
        if (__any(flo || fhi)) {
#pragma unroll
          for (int u = 0; u < KGR; ++u) {
            um[u] = flo ? u0[u] : (F)0;
            up[u] = fhi ? u0[u] : (F)0;
          }
          prod_acc<P, NC, KGR, NCB>(acc, Cf + 3 * bstride + kg * gstride, um);
          prod_acc<P, NC, KGR, NCB>(acc, Cf + 4 * bstride + kg * gstride, up);
        }
      }
      // the neighbours' face rows
      if (__any(flo)) {
        const int pn = face_cell(d, axis, true, f);
        for (int kg = 0; kg < kgl; ++kg) {
          F gn[KGR];
#pragma unroll
          for (int u = 0; u < KGR; ++u) {
            const int kc = 32 * kg + sub_col<P>(u, kq);
            const bool in = flo && lo >= 0 && kc < rl;
            const double v = Ul[(int64_t)(in ? kc : 0) * N + pn];
            gn[u] = in ? (F)v : (F)0;
          }
          prod_acc<P, NC, KGR, NCB>(acc, Cf + 5 * bstride + kg * gstride, gn);
        }
      }
      if (__any(fhi)) {
        const int pn = face_cell(d, axis, false, f);
        for (int kg = 0; kg < kgh; ++kg) {
          F gn[KGR];
#pragma unroll
          for (int u = 0; u < KGR; ++u) {
            const int kc = 32 * kg + sub_col<P>(u, kq);
            const bool in = fhi && hi >= 0 && kc < rh;
            const double v = Uh[(int64_t)(in ? kc : 0) * N + pn];
            gn[u] = in ? (F)v : (F)0;
          }
          prod_acc<P, NC, KGR, NCB>(acc, Cf + 6 * bstride + kg * gstride, gn);
        }
      }
#pragma unroll
      for (int cb = 0; cb < NC; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = c0 + out_col<P>(cb, v, kq);
          if (rin && j < t) K1[(int64_t)j * N + p] = (S)acc[cb][v];
        }
    }
  };
  constexpr int KG1 = P == 2 ? 8 : 4;
  const int rmax = max(r, max(rl, rh));
  if (live_sub<P>(rmax) <= KG1 && t - c0 <= 16) run(wint<KG1>{}, wint<1>{});
  else run(wint<KG>{}, wint<NCB>{});
}

// L-step of an advection stage (eq. advx_evolL), weighted by sqrt(w), for
// output columns [c0, c0 + 32):
//   AL[q,:] = Qh[q,:] P0 + Omega_q^+ Qh[q,:] Pm + Omega_q^- Qh[q,:] Pp,
// with one accumulator set per coefficient matrix and the per-direction
// factors applied to the accumulators (each lane's accumulators belong to
// its own direction).
template <class S, int P, int NM, int NCB>
__global__ __launch_bounds__(WTHR) void kw_lstep(Dev d, int axis, int sd0) {
  using F = typename Prec<P>::F;
  using Acc = typename Prec<P>::Acc;
  static_assert(NM == 3 || NM == 9, "Euler (P0, Pm, Pp) or RK4 (P0, N1..N4 of each class)");
  constexpr int NG = WCAP_T / 64;
  constexpr int gstride = 16 * NCB * 64;         // one group of one matrix
  const int s = sd0 + blockIdx.y;
  const int t = d.tdim[s];
  const int c0 = blockIdx.z * 16 * NCB;
  if (c0 >= t) return;
  const int M = d.M, T = d.T;
  const int ng = wdiv(t, 64);
  const double* om = axis == 0 ? d.omx : d.omy;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  extern __shared__ double lds[];
  F* Pf = reinterpret_cast<F*>(lds);  // [m][g] groups
  {
    const double* sm = small_of(d, s);
    int offs[NM];
    offs[0] = d.oP0;
    if (NM == 3) {
      offs[1] = d.oPm;
      offs[2] = d.oPp;
    } else {
      const int op[4] = {d.oPm, d.oW1, d.oW3, d.oW5}, on[4] = {d.oPp, d.oW2, d.oW4, d.oW6};
      for (int j = 0; j < 4; ++j) {
        offs[1 + j] = op[j];
        offs[5 + j] = on[j];
      }
    }
    const int total = NM * NG * gstride;
    for (int idx = threadIdx.x; idx < total; idx += WTHR) {
      const int l = idx & 63, f = idx >> 6, cb = f % NCB, u = (f / NCB) % 16, g = (f / (16 * NCB)) % NG,
                m = f / (16 * NCB * NG);
      const int kc = 64 * g + sub_col<P>(u, l >> 4), col = c0 + 16 * cb + (l & 15);
      Pf[idx] = (kc < t && col < t) ? (F)sm[offs[m] + kc + col * T] : (F)0;
    }
  }
  __syncthreads();
  const S* Qsd = (const S*)d.Qh + (int64_t)s * M * T;
  S* ALs = (S*)d.AL + (int64_t)s * M * T;
  const int nst = wdiv(M, 16);
  const int stride = gridDim.x * WNW;
  // NS sub-steps of each 64-column group and NC output column blocks are
  // issued: a subdomain with one short group and at most 16 live columns in
  // the block takes the short instance
  auto run = [&](auto ns_c, auto nc_c) {
    constexpr int NS = decltype(ns_c)::value, NC = decltype(nc_c)::value;
    F xv[NS], xn[NS];
    auto load = [&](int st_, int g_) {
      const int q_ = st_ * 16 + l16;
      const int qc = q_ < M ? q_ : M - 1;
#pragma unroll
      for (int u = 0; u < NS; ++u) {
        const int kc = 64 * g_ + sub_col<P>(u, kq);
        const bool in = q_ < M && kc < t;
        const S v = Qsd[(int64_t)(in ? kc : 0) * M + qc];
        xn[u] = in ? (F)v : (F)0;
      }
    };
    int st = blockIdx.x * WNW + wave, g = 0;
    if (st < nst) load(st, 0);
    Acc a[NM][NC];
#pragma unroll
    for (int m = 0; m < NM; ++m) zero_prod<P>(a[m], NC);
    while (st < nst) {
#pragma unroll
      for (int u = 0; u < NS; ++u) xv[u] = xn[u];
      int st2 = st, g2 = g + 1;
      if (g2 >= ng) {
        g2 = 0;
        st2 = st + stride;
      }
      if (st2 < nst) load(st2, g2);
#pragma unroll
      for (int m = 0; m < NM; ++m) prod_acc<P, NC, NS, NCB>(a[m], Pf + (m * NG + g) * gstride, xv);
      if (g == ng - 1) {
        const int q = st * 16 + l16;
        const bool rin = q < M;
        const double o = rin ? om[q] : 0.0;
        const double op = o >= 0.0 ? o : 0.0, on = o < 0.0 ? o : 0.0;
#pragma unroll
        for (int cb = 0; cb < NC; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int j = c0 + out_col<P>(cb, v, kq);
            double val;
            if (NM == 3) {
              val = (double)a[0][cb][v] + op * (double)a[1][cb][v] + on * (double)a[2][cb][v];
            } else {
              // sum_j w^j N_j of the direction's class, nested in w
              double vp = (double)a[4][cb][v], vn = (double)a[8][cb][v];
#pragma unroll
              for (int m = 3; m >= 1; --m) {
                vp = fma(vp, op, (double)a[m][cb][v]);
                vn = fma(vn, on, (double)a[4 + m][cb][v]);
              }
              val = (double)a[0][cb][v] + op * vp + on * vn;
            }
            if (rin && j < t) ALs[(int64_t)j * M + q] = (S)val;
          }
#pragma unroll
        for (int m = 0; m < NM; ++m) zero_prod<P>(a[m], NC);
      }
      st = st2;
      g = g2;
    }
  };
  constexpr int NS1 = P == 2 ? 8 : 4;
  if (ng == 1 && live_sub<P>(t) <= NS1 && t - c0 <= 16) run(wint<NS1>{}, wint<1>{});
  else run(wint<16>{}, wint<NCB>{});
}

// Degree-4 Taylor polynomial of exp: e(y) = 1 + y + y^2/2 + y^3/6 + y^4/24,
// and the divided difference (e(x) - e(y)) / (x - y) of e(dt .) written
// without the division (x = dt a, y = dt b; the result carries the factor dt).
__device__ __forceinline__ double taylor_e4(double y) {
  return 1.0 + y * (1.0 + y * (0.5 + y * (1.0 / 6.0 + y * (1.0 / 24.0))));
}
__device__ __forceinline__ double taylor_d4(double x, double y, double dt) {
  const double s1 = x + y, s2 = x * x + x * y + y * y, s3 = x * x * x + x * x * y + x * y * y + y * y * y;
  return dt * (1.0 + 0.5 * s1 + s2 * (1.0 / 6.0) + s3 * (1.0 / 24.0));
}

// RK4 substeps of the advection K-step (Algorithms 1-2, step 1, with the
// classic four-stage method; Section 4).  The right-hand side
//   g(K) = -(c / h) [ (K - K_prev) C+ + (K_next - K) C- ]
// is affine in K once the ghost rows K^b of the faces are frozen, so one
// RK4 step equals the nested form
//   K1 = K0 + dt g(K0 + dt/2 g(K0 + dt/3 g(K0 + dt/4 g(K0)))),
// four passes of "out = K0 + alpha g(in)" over the materialised arrays.
//
// One nested stage: out = K0 + alpha g(in) for output columns [c0, c0 + 32)
// of one tile of 64 cells (FP64).  A thread owns one cell and four columns;
// C+ and C- (columns c0..c0+31, all t rows) sit in LDS.
constexpr int RKC = 32;  // output columns per workgroup
__global__ __launch_bounds__(WTHR) void kw_rk_kstep(Dev d, int axis, int sd0, double alpha, const double* in,
                                                    double* out) {
  const int s = sd0 + blockIdx.y;
  const int t = d.tdim[s];
  const int c0 = blockIdx.z * RKC;
  if (c0 >= t) return;
  const int N = d.N, T = d.T;
  __shared__ double Cps[WCAP_T * RKC], Cns[WCAP_T * RKC];
  const double* sm = small_of(d, s);
  for (int idx = threadIdx.x; idx < t * RKC; idx += WTHR) {
    const int k = idx / RKC, c = idx % RKC, j = c0 + c;
    Cps[idx] = j < t ? sm[d.oCp + k + j * T] : 0.0;
    Cns[idx] = j < t ? sm[d.oCn + k + j * T] : 0.0;
  }
  __syncthreads();
  const int p = blockIdx.x * 64 + (threadIdx.x & 63);
  if (p >= N) return;
  const int cg = (threadIdx.x >> 6) * 4;  // this thread's first column in the block
  const int ix = p % d.lnx, iy = p / d.lnx;
  const int pos = axis == 0 ? ix : iy, len = axis == 0 ? d.lnx : d.lny, f = axis == 0 ? iy : ix;
  const int step = axis == 0 ? 1 : d.lnx;
  const double* K0 = d.K3 + (int64_t)s * N * T;
  const double* X = in + (int64_t)s * N * T;
  double* Y = out + (int64_t)s * N * T;
  const double* glo = d.ghost + (int64_t)(2 * s) * T * d.face;
  const double* ghi = glo + (int64_t)T * d.face;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < t; ++k) {
    const double x = X[(int64_t)k * N + p];
    const double xp = pos > 0 ? X[(int64_t)k * N + p - step] : glo[(int64_t)k * d.face + f];
    const double xn = pos < len - 1 ? X[(int64_t)k * N + p + step] : ghi[(int64_t)k * d.face + f];
    const double dm = x - xp, dp = xn - x;
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = fma(dm, Cps[k * RKC + cg + c], fma(dp, Cns[k * RKC + cg + c], acc[c]));
  }
  const double sc = -alpha * d.c / d.h;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int j = c0 + cg + c;
    if (j < t) Y[(int64_t)j * N + p] = fma(sc, acc[c], K0[(int64_t)j * N + p]);
  }
}

// Collision K-step (eq. coll_evolK) for output columns [c0, c0 + 32), with
// K = U S and m = V^T w:
//   K1[p] = (1 - dt c_t[p]) K[p] + dt (c_s[p] / W (K[p].m) + Q[p]) m;
// K[p].m = U[p] (S m) is an extra product block.  With RK4 substeps the
// row ODE K' = K (a m m^T - b I) + Q m^T (a = c_s / W, b = c_t) has the
// degree-4 Taylor step
//   K1 = e(-b) K + (a D(lam, -b) (K.m) + Q D(lam, 0)) m,  lam = -b + a m.m,
// with e(x) = sum_{j <= 4} (dt x)^j / j! and D(x, y) = (e(x) - e(y)) / (x - y)
// (the rank-one part of the matrix power collapses because m m^T m = (m.m) m).
template <class S, int P>
__global__ __launch_bounds__(WTHR) void kw_coll_kstep(Dev d, int sd0) {
  using F = typename Prec<P>::F;
  using Acc = typename Prec<P>::Acc;
  constexpr int NCB = 2, KSP = 16;
  const int s = sd0 + blockIdx.y;
  const int r = d.rank[s];
  const int c0 = blockIdx.z * 16 * NCB;
  if (c0 >= r) return;
  const int N = d.N, R = d.R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  __shared__ double mv[WCAP_R], smv[WCAP_R];
  __shared__ F Bf[KSP * NCB * 64];
  __shared__ F Be[KSP * 64];
  const double* sm = small_of(d, s);
  const double* Sg = d.S + (int64_t)s * R * R;
  for (int a = threadIdx.x; a < WCAP_R; a += WTHR) mv[a] = a < r ? sm[d.oMv + a] : 0.0;
  __syncthreads();
  for (int a = threadIdx.x; a < WCAP_R; a += WTHR) {
    double acc = 0.0;
    for (int b = 0; b < r; ++b) acc = fma(Sg[a + b * R], mv[b], acc);
    smv[a] = a < r ? acc : 0.0;
  }
  double mu = 0.0;  // m.m (RK4 only)
  if (d.rk4)
    for (int b = 0; b < r; ++b) mu = fma(mv[b], mv[b], mu);
  for (int idx = threadIdx.x; idx < KSP * NCB * 64; idx += WTHR) {
    const int l = idx & 63, f = idx >> 6, cb = f % NCB, u = f / NCB;
    const int kc = sub_col<P>(u, l >> 4), col = c0 + 16 * cb + (l & 15);
    Bf[idx] = (kc < r && col < r) ? (F)Sg[kc + col * R] : (F)0;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < KSP * 64; idx += WTHR) {
    const int l = idx & 63, u = idx >> 6;
    const int kc = sub_col<P>(u, l >> 4), col = l & 15;
    Be[idx] = (kc < r && col == 0) ? (F)smv[kc] : (F)0;
  }
  __syncthreads();
  const double* Us = d.U + (int64_t)s * N * R;
  const double* cs = d.cs + (int64_t)s * N;
  const double* ct = d.ct + (int64_t)s * N;
  const double* Qs = d.Qsrc + (int64_t)s * N;
  S* K1 = (S*)d.K1 + (int64_t)s * N * d.T;
  const double dt = d.dt, iW = 1.0 / d.W;
  const int nst = wdiv(N, 16);
  const int stride = gridDim.x * WNW;
  // a subdomain of rank <= 16 (one short group, one column block) takes the
  // short instance
  auto run = [&](auto ns_c, auto nc_c) {
    constexpr int NS = decltype(ns_c)::value, NC = decltype(nc_c)::value;
    F xn[NS];
    auto load = [&](int st_) {
      const int p_ = st_ * 16 + l16;
      const int pc = p_ < N ? p_ : N - 1;
#pragma unroll
      for (int u = 0; u < NS; ++u) {
        const int kc = sub_col<P>(u, kq);
        const bool in = p_ < N && kc < r;
        const double v = Us[(int64_t)(in ? kc : 0) * N + pc];
        xn[u] = in ? (F)v : (F)0;
      }
    };
    int st = blockIdx.x * WNW + wave;
    if (st < nst) load(st);
    for (; st < nst; st += stride) {
      F xv[NS];
#pragma unroll
      for (int u = 0; u < NS; ++u) xv[u] = xn[u];
      if (st + stride < nst) load(st + stride);
      const int p = st * 16 + l16;
      const bool rin = p < N;
      const int pc = rin ? p : N - 1;
      Acc acc[NC], ae[1];
      zero_prod<P>(acc, NC);
      zero_prod<P>(ae, 1);
      prod_acc<P, NC, NS, NCB>(acc, Bf, xv);
      prod_acc<P, 1, NS>(ae, Be, xv);
      // column 0 of the extra block sits in component 0 of lanes 0..15
      const double km = __shfl((double)ae[0][0], l16, 64);
      double a0, a1;
      if (!d.rk4) {
        a0 = rin ? 1.0 - dt * ct[pc] : 0.0;
        a1 = rin ? dt * (cs[pc] * iW * km + Qs[pc]) : 0.0;
      } else {
        const double b = ct[pc], aa = cs[pc] * iW;
        const double yb = -dt * b, yl = dt * (aa * mu - b);
        a0 = rin ? taylor_e4(yb) : 0.0;
        a1 = rin ? aa * taylor_d4(yl, yb, dt) * km + Qs[pc] * taylor_d4(yl, 0.0, dt) : 0.0;
      }
#pragma unroll
      for (int cb = 0; cb < NC; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = c0 + out_col<P>(cb, v, kq);
          if (rin && j < r) K1[(int64_t)j * N + p] = (S)fma(a0, (double)acc[cb][v], a1 * mv[j]);
        }
    }
  };
  constexpr int NS1 = P == 2 ? 8 : 4;
  if (live_sub<P>(r) <= NS1 && r - c0 <= 16) run(wint<NS1>{}, wint<1>{});
  else run(wint<KSP>{}, wint<NCB>{});
}

// ----------------------------------------------------------------------------
// Reductions over rows: for each job and each 64 x 64 block (a, b),
//   out[64 a + i, 64 b + j] = scale sum_rows w(row) X[row, 64 a + i] Y'[row, 64 b + j]
// where Y' is Y, or Y[p + e] - Y[p] (zero beyond the high face) for the
// spatial Galerkin matrix.  blockIdx.z enumerates (job, block); each
// workgroup writes its block of its own partial.  Symmetric jobs form the
// blocks with a <= b and store each entry and its mirror (a diagonal block
// only from i <= j), so the sum comes out exactly symmetric.
// ----------------------------------------------------------------------------
__device__ __forceinline__ int src_subdomain(const Dev& d, int s, int axis, int side) {
  return side == 0 ? s : neighbour(d, s, axis, side);
}

__device__ __forceinline__ int src_cols(const Dev& d, int s, int axis, const XSrc& x) {
  if (x.vec) return 1;
  const int sd = src_subdomain(d, s, axis, x.side);
  if (sd < 0) return 0;
  return x.side == 0 ? dim_of(d, s, axis, x.dim) : d.rank[sd];
}

// cell / direction index of row `row` of a source (rows are face entries for
// face sources; the neighbour's face is the one touching this subdomain)
__device__ __forceinline__ int src_row(const Dev& d, int axis, const XSrc& x, int row) {
  if (x.face == 0) return row;
  return face_cell(d, axis, x.face == 2, row);
}

template <class W>
__device__ __forceinline__ double src_load(const Dev& d, int s, int axis, const XSrc& x, int row, int col) {
  const int sd = src_subdomain(d, s, axis, x.side);
  const int64_t base = (int64_t)(sd < 0 ? 0 : sd) * x.sd;
  const int pr = src_row(d, axis, x, row);
  double v;
  if (x.vec) v = ((const double*)x.p)[base + pr];
  else if (x.is64) v = ((const double*)x.p)[base + (int64_t)col * x.ld + pr];
  else v = (double)((const W*)x.p)[base + (int64_t)col * x.ld + pr];
  if (x.rowscale) v *= d.sw[pr];
  return v;
}

template <class W>
__global__ __launch_bounds__(XTHR, 4) void kw_xgram(Dev d, int axis, int sd0, XJobs jobs) {
  const int s = sd0 + blockIdx.y;
  if (jobs.skip_off >= 0 && small_of(d, s)[jobs.skip_off] != 0.0) return;
  int jb = 0;
#pragma unroll
  for (int q = 1; q < XJOBS_MAX; ++q)
    if (q < jobs.n && (int)blockIdx.z >= jobs.j[q].zbase) jb = q;
  // a runtime index into the job array would place it in scratch memory:
  // copy the selected job out with static indices
  XJob J = jobs.j[0];
#pragma unroll
  for (int q = 1; q < XJOBS_MAX; ++q)
    if (q == jb) J = jobs.j[q];
  int pz = blockIdx.z - J.zbase, a, b;
  if (J.sym) {
    b = 0;
    while (pz > b) {
      pz -= b + 1;
      ++b;
    }
    a = pz;
  } else {
    a = pz % J.pa;
    b = pz / J.pa;
  }
  const int nx = src_cols(d, s, axis, J.x), ny = src_cols(d, s, axis, J.y);
  const bool live = 64 * a < nx && 64 * b < ny;
  if (!live) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  // a chunk of XR rows of the 64 X columns and 64 Y columns of the block,
  // column-major in LDS (odd leading dimension); the loads put consecutive
  // lanes on consecutive rows of one column
  constexpr int XR = 32, XLD = XR + 1;
  __shared__ double xs[64 * XLD], ys[64 * XLD];
  const int rows = J.rows_cells ? (J.x.face ? face_len(d, axis) : d.N) : d.M;
  const double* om = axis == 0 ? d.omx : d.omy;
  const double* wcell = J.wmode == 4 ? d.cs + (int64_t)s * d.N : d.ct + (int64_t)s * d.N;
  const int e = axis == 0 ? 1 : d.lnx;
  const int na = axis == 0 ? d.lnx : d.lny;
  // per-source constants
  const int sdx = src_subdomain(d, s, axis, J.x.side), sdy = src_subdomain(d, s, axis, J.y.side);
  const int64_t bx = (int64_t)(sdx < 0 ? 0 : sdx) * J.x.sd, by = (int64_t)(sdy < 0 ? 0 : sdy) * J.y.sd;
  const int cx0 = 64 * a, cy0 = 64 * b;
  // thread (wave, lane) loads row lane % 32 of the columns 2 (8 wave + q) +
  // lane / 32 (q < 8) of the chunk, for X and for Y
  constexpr int NQ = 64 * XR / XTHR;
  const int lr = lane % XR, lc = lane / XR;  // XR = 32: two columns per load instruction
  const double* xd = (const double*)J.x.p + bx;
  const W* xw = (const W*)J.x.p + bx;
  const double* yd = (const double*)J.y.p + by;
  const W* yw = (const W*)J.y.p + by;
  // columns cb0 + 2 q + lane / 32 (q < NQ) of rows ch XR + lane % 32
  auto fetch = [&](int ch, int cb0, double (&xv)[NQ], double (&yv)[NQ]) {
    const int row = ch * XR + lr;
    const bool rin = row < rows;
    const int rc = rin ? row : 0;
    double wt = rin ? 1.0 : 0.0;
    if (J.wmode == 1) wt *= om[rc];
    else if (J.wmode == 2) wt *= om[rc] >= 0.0 ? 1.0 : 0.0;
    else if (J.wmode == 3) wt *= om[rc] < 0.0 ? 1.0 : 0.0;
    else if (J.wmode >= 4) wt *= wcell[rc];
    const int px = src_row(d, axis, J.x, rc), py = src_row(d, axis, J.y, rc);
    bool hs = false;
    if (J.shift) {
      const int ia = axis == 0 ? rc % d.lnx : rc / d.lnx;
      hs = ia < na - 1;
    }
    const double sx = J.x.rowscale ? d.sw[px] : 1.0, sy = J.y.rowscale ? d.sw[py] : 1.0;
    const double sy1 = (J.shift && J.y.rowscale) ? d.sw[hs ? py + e : py] : sy;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int cl = cb0 + 2 * q + lc;  // column of the block, 0..63
      const int ci = cx0 + cl, cj = cy0 + cl;
      const bool xin = ci < nx, yin = cj < ny;
      double v = 0.0, u = 0.0;
      // offsets within a subdomain's slab fit in 32 bits: the loads take the
      // slab base as a scalar and a 32-bit offset per lane
      if (xin && wt != 0.0) {
        const unsigned ox = J.x.vec ? (unsigned)px : (unsigned)(ci * J.x.ld + px);
        v = (J.x.vec || J.x.is64) ? xd[ox] : (double)xw[ox];
        v = v * sx * wt;
      }
      if (yin && rin) {
        const unsigned oy = J.y.vec ? (unsigned)py : (unsigned)(cj * J.y.ld + py);
        const bool w64 = J.y.vec || J.y.is64;
        u = w64 ? yd[oy] : (double)yw[oy];
        u *= sy;
        if (J.shift) {
          double u1 = 0.0;
          if (hs) u1 = (w64 ? yd[oy + e] : (double)yw[oy + e]) * sy1;
          u = u1 - u;
        }
      }
      xv[q] = v;
      yv[q] = u;
    }
  };
  auto stash = [&](double* xb, double* yb, int cb0, const double (&xv)[NQ], const double (&yv)[NQ]) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int cl = cb0 + 2 * q + lc;
      xb[cl * XLD + lr] = xv[q];
      yb[cl * XLD + lr] = yv[q];
    }
  };
  const int nch = wdiv(rows, XR);
  if (nx - cx0 <= 16 && ny - cy0 <= 16) {
    // a block with at most 16 live rows and columns: each wavefront stages
    // and reduces chunks of its own (32 rows of 16 columns, no workgroup
    // barrier), then the four sums are added in a fixed order
    constexpr int XNW = XTHR / 64;
    double* xw = xs + wave * 16 * XLD;
    double* yw = ys + wave * 16 * XLD;
    dbl4 acc = zero4();
    for (int ch = blockIdx.x * XNW + wave; ch < nch; ch += gridDim.x * XNW) {
      {
        double xv[NQ], yv[NQ];
        fetch(ch, 0, xv, yv);
        stash(xw, yw, 0, xv, yv);
      }
      wave_sync();
      const double* xa = xw + l16 * XLD + kq;
      const double* yb = yw + l16 * XLD + kq;
      dbl4 cacc = zero4();
#pragma unroll
      for (int ks = 0; ks < XR / 4; ++ks) cacc = mfma64(xa[4 * ks], yb[4 * ks], cacc);
      acc += cacc;
      wave_sync();
    }
    __syncthreads();
    double* red = xs;
#pragma unroll
    for (int v = 0; v < 4; ++v) red[(wave * 4 + v) * 64 + lane] = acc[v];
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double tot = red[v * 64 + lane];
#pragma unroll
      for (int w = 1; w < XNW; ++w) tot += red[(w * 4 + v) * 64 + lane];
      acc[v] = tot;
    }
    double* out = gpart_of(d, s) + (int64_t)blockIdx.x * d.gpTile + J.out_off;
    const int ld = J.out_ld > 0 ? J.out_ld : nx;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 64 * a + 4 * v + kq, j = 64 * b + l16;
      if (i >= nx || j >= ny) continue;
      const double val = J.scale * acc[v];
      if (J.sym) {
        if (a == b && i > j) continue;
        out[i + (int64_t)j * ld] = val;
        out[j + (int64_t)i * ld] = val;
      } else {
        out[i + (int64_t)j * ld] = val;
      }
    }
    return;
  }
  // wavefront w accumulates the output rows 16 w .. 16 w + 15 of the block,
  // in NCJ column blocks of 16 (only as many as the block has live columns);
  // a wavefront whose rows are all beyond the live ones only stages data
  const bool wlive = cx0 + 16 * wave < nx;
  auto run = [&](auto ncj_c) {
    constexpr int NCJ = decltype(ncj_c)::value;
    dbl4 acc[NCJ];
    zero_acc<NCJ>(acc);
    for (int ch = blockIdx.x; ch < nch; ch += gridDim.x) {
      {
        double xv[NQ], yv[NQ];
        fetch(ch, 2 * NQ * wave, xv, yv);
        __syncthreads();
        stash(xs, ys, 2 * NQ * wave, xv, yv);
      }
      __syncthreads();
      if (wlive) {
        const double* xa = xs + (16 * wave + l16) * XLD + kq;
        const double* yb = ys + l16 * XLD + kq;
        // each chunk is summed on its own and then added to the running
        // total, so no chain of roundings runs over more than one chunk (the
        // angular sums cancel strongly near sources)
        dbl4 cacc[NCJ];
        zero_acc<NCJ>(cacc);
#pragma unroll
        for (int ks = 0; ks < XR / 4; ++ks) {
          const double av = xa[4 * ks];
#pragma unroll
          for (int cj = 0; cj < NCJ; ++cj) cacc[cj] = mfma64(av, yb[16 * cj * XLD + 4 * ks], cacc[cj]);
        }
#pragma unroll
        for (int cj = 0; cj < NCJ; ++cj) acc[cj] += cacc[cj];
      }
    }
    if (!wlive) return;
    double* out = gpart_of(d, s) + (int64_t)blockIdx.x * d.gpTile + J.out_off;
    const int ld = J.out_ld > 0 ? J.out_ld : nx;
#pragma unroll
    for (int cj = 0; cj < NCJ; ++cj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 64 * a + 16 * wave + 4 * v + kq, j = 64 * b + 16 * cj + l16;
        if (i >= nx || j >= ny) continue;
        const double val = J.scale * acc[cj][v];
        if (J.sym) {
          if (a == b && i > j) continue;
          out[i + (int64_t)j * ld] = val;
          out[j + (int64_t)i * ld] = val;
        } else {
          out[i + (int64_t)j * ld] = val;
        }
      }
  };
  const int ncj = ny - cy0;
  if (ncj <= 16) run(wint<1>{});
  else if (ncj <= 32) run(wint<2>{});
  else run(wint<4>{});
}

// ============================================================================
// small kernels: building blocks for 1024-thread workgroups
// ============================================================================

// sum over the workgroup in a fixed order (red: SNW doubles of LDS)
__device__ __forceinline__ double s_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += red[w];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double s_max(double v, double* red) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, red[w]);
  __syncthreads();
  return r;
}

// acc[u] = sum over the ngp partials, added in order w = 0, 1, ..., of
// gp[w tile + src[u]], for UI entries at once: each group of four partials
// issues all 4 UI loads before the first addition, so one workgroup keeps
// enough loads in flight to cover the memory latency
template <int UI>
__device__ __forceinline__ void sum_partials_multi(const double* gp, int64_t tile, int ngp, const int64_t (&src)[UI],
                                                   double (&acc)[UI]) {
#pragma unroll
  for (int u = 0; u < UI; ++u) acc[u] = 0.0;
  int w = 0;
  for (; w + 4 <= ngp; w += 4) {
    double v[4][UI];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int u = 0; u < UI; ++u) v[a][u] = gp[(int64_t)(w + a) * tile + src[u]];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int u = 0; u < UI; ++u) acc[u] += v[a][u];
  }
  for (; w < ngp; ++w)
#pragma unroll
    for (int u = 0; u < UI; ++u) acc[u] += gp[(int64_t)w * tile + src[u]];
}

// dst (rows x cols, ldd) = scale * sum over ngp partials of the block at off
// (leading dimension ldp), partials added in a fixed order
__device__ void s_sum_partials(const Dev& d, int s, int ngp, int off, int ldp, int rows, int cols, double* dst,
                               int ldd, double scale) {
  constexpr int UI = 4;
  const double* gp = gpart_of(d, s);
  const int total = rows * cols;
  for (int base = threadIdx.x; base < total; base += UI * STHR) {  // STHR-thread kernels only
    int64_t src[UI];
#pragma unroll
    for (int u = 0; u < UI; ++u) {
      const int idx = base + u * STHR;
      const int i = idx % rows, j = idx / rows;
      src[u] = idx < total ? off + i + (int64_t)j * ldp : off;
    }
    double acc[UI];
    sum_partials_multi<UI>(gp, d.gpTile, ngp, src, acc);
#pragma unroll
    for (int u = 0; u < UI; ++u) {
      const int idx = base + u * STHR;
      if (idx < total) dst[idx % rows + (int64_t)(idx / rows) * ldd] = scale * acc[u];
    }
  }
}

// C (m x n, ldc) = alpha op(A) op(B) + beta D on the FP64 matrix cores, any
// pointers (LDS or global), C aliasing neither A nor B; the 16 x 16 output
// tiles are dealt to the wavefronts, k walked in steps of 64 with all operand
// loads of a step issued first.  Ends with a barrier.
__device__ __forceinline__ void gmm_t1(double* C, int ldc, const double* A, int lda, bool ta, const double* B,
                                       int ldb, bool tb, int m, int n, int k, double alpha, double beta,
                                       const double* D, int ldd) {
  constexpr int KC = 16, NL = KC / 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int nw = SNW;  // called by STHR-thread kernels only
  const int l16 = lane & 15, kq = lane >> 4;
  const int tm = wdiv(m, 16), tn = wdiv(n, 16);
  const int nch = wdiv(k, KC);
  for (int tile = wave; tile < tm * tn; tile += nw) {
    const int ti = tile % tm, tj = tile / tm;
    const int i0 = 16 * ti, j0 = 16 * tj;
    const int i = i0 + l16, j = j0 + l16;
    const int ic = i < m ? i : 0, jc = j < n ? j : 0;
    // operands of the next 16 values of k are loaded while the MFMAs of
    // the current ones run
    auto load = [&](int c, double (&av)[NL], double (&bv)[NL]) {
#pragma unroll
      for (int u = 0; u < NL; ++u) {
        const int l = c * KC + 4 * u + kq;
        const int lc = l < k ? l : 0;
        const double a_ = ta ? A[lc + (int64_t)ic * lda] : A[ic + (int64_t)lc * lda];
        const double b_ = tb ? B[jc + (int64_t)lc * ldb] : B[lc + (int64_t)jc * ldb];
        av[u] = (i < m && l < k) ? a_ : 0.0;
        bv[u] = (j < n && l < k) ? b_ : 0.0;
      }
    };
    dbl4 e = zero4(), o = zero4();
    double a0[NL], b0[NL], a1[NL], b1[NL];
    if (nch > 0) load(0, a0, b0);
    for (int c = 0; c < nch; c += 2) {
      if (c + 1 < nch) load(c + 1, a1, b1);
#pragma unroll
      for (int u = 0; u < NL; u += 2) {
        e = mfma64(a0[u], b0[u], e);
        o = mfma64(a0[u + 1], b0[u + 1], o);
      }
      if (c + 1 >= nch) break;
      if (c + 2 < nch) load(c + 2, a0, b0);
#pragma unroll
      for (int u = 0; u < NL; u += 2) {
        e = mfma64(a1[u], b1[u], e);
        o = mfma64(a1[u + 1], b1[u + 1], o);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ci = i0 + 4 * v + kq, cj = j0 + l16;
      if (ci < m && cj < n) {
        const double acc = e[v] + o[v];
        C[ci + (int64_t)cj * ldc] = beta == 0.0 ? alpha * acc : fma(alpha, acc, beta * D[ci + (int64_t)cj * ldd]);
      }
    }
  }
  __syncthreads();
}

// The same product with 2 x 2 output tiles per wavefront and step: the
// operands of two row blocks and two column blocks are loaded once for four
// tiles (half the loads per matrix-core instruction), k walked in steps of 4
// with the next step's operands loaded while the current MFMAs run.
template <bool ta, bool tb>
__device__ __forceinline__ void gmm_t2(double* C, int ldc, const double* A, int lda, const double* B, int ldb, int m,
                                       int n, int k, double alpha, double beta, const double* D, int ldd) {
  constexpr int KC = 4, NL = KC / 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int nw = SNW;  // called by STHR-thread kernels only
  const int l16 = lane & 15, kq = lane >> 4;
  const int bm = wdiv(m, 32), bn = wdiv(n, 32);
  const int nch = wdiv(k, KC);
  for (int blk = wave; blk < bm * bn; blk += nw) {
    const int i0 = 32 * (blk % bm), j0 = 32 * (blk / bm);
    int ic[2], jc[2];
    bool iv[2], jv[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const int i = i0 + 16 * x + l16, j = j0 + 16 * x + l16;
      iv[x] = i < m;
      jv[x] = j < n;
      ic[x] = iv[x] ? i : 0;
      jc[x] = jv[x] ? j : 0;
    }
    auto load = [&](int c, double (&av)[2][NL], double (&bv)[2][NL]) {
#pragma unroll
      for (int u = 0; u < NL; ++u) {
        const int l = c * KC + 4 * u + kq;
        const bool lin = l < k;
        const int lc = lin ? l : 0;
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          const double a_ = ta ? A[lc + (int64_t)ic[x] * lda] : A[ic[x] + (int64_t)lc * lda];
          const double b_ = tb ? B[jc[x] + (int64_t)lc * ldb] : B[lc + (int64_t)jc[x] * ldb];
          av[x][u] = (iv[x] && lin) ? a_ : 0.0;
          bv[x][u] = (jv[x] && lin) ? b_ : 0.0;
        }
      }
    };
    dbl4 acc[2][2] = {{zero4(), zero4()}, {zero4(), zero4()}};
    double a0[2][NL], b0[2][NL], a1[2][NL], b1[2][NL];
    if (nch > 0) load(0, a0, b0);
    for (int c = 0; c < nch; c += 2) {
      if (c + 1 < nch) load(c + 1, a1, b1);
#pragma unroll
      for (int u = 0; u < NL; ++u)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) acc[x][y] = mfma64(a0[x][u], b0[y][u], acc[x][y]);
      if (c + 1 >= nch) break;
      if (c + 2 < nch) load(c + 2, a0, b0);
#pragma unroll
      for (int u = 0; u < NL; ++u)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) acc[x][y] = mfma64(a1[x][u], b1[y][u], acc[x][y]);
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ci = i0 + 16 * x + 4 * v + kq, cj = j0 + 16 * y + l16;
          if (ci < m && cj < n) {
            const double a = acc[x][y][v];
            C[ci + (int64_t)cj * ldc] = beta == 0.0 ? alpha * a : fma(alpha, a, beta * D[ci + (int64_t)cj * ldd]);
          }
        }
  }
  __syncthreads();
}

// products of at least 2 SNW tiles take the 2 x 2 tiling
__device__ void gmm(double* C, int ldc, const double* A, int lda, bool ta, const double* B, int ldb, bool tb, int m,
                    int n, int k, double alpha, double beta, const double* D, int ldd) {
  if (wdiv(m, 16) * wdiv(n, 16) >= 2 * SNW) {
    if (ta && tb) gmm_t2<true, true>(C, ldc, A, lda, B, ldb, m, n, k, alpha, beta, D, ldd);
    else if (ta) gmm_t2<true, false>(C, ldc, A, lda, B, ldb, m, n, k, alpha, beta, D, ldd);
    else if (tb) gmm_t2<false, true>(C, ldc, A, lda, B, ldb, m, n, k, alpha, beta, D, ldd);
    else gmm_t2<false, false>(C, ldc, A, lda, B, ldb, m, n, k, alpha, beta, D, ldd);
  } else
    gmm_t1(C, ldc, A, lda, ta, B, ldb, tb, m, n, k, alpha, beta, D, ldd);
}

__device__ __forceinline__ void gmm(double* C, int ldc, const double* A, int lda, bool ta, const double* B, int ldb,
                                    bool tb, int m, int n, int k, double alpha, double beta) {
  gmm(C, ldc, A, lda, ta, B, ldb, tb, m, n, k, alpha, beta, C, ldc);
}

// C = alpha A B + beta D for n x n matrices whose product is symmetric (A,
// B, D symmetric, A and B commuting, as for polynomials in one symmetric
// matrix): only the 16 x 16 tiles on and above the diagonal are formed and
// each value is stored at (i, j) and (j, i) (in a diagonal tile only i <= j
// writes), so C comes out exactly symmetric and iterations built on it keep
// exact symmetry.  B is read by rows (B[l][j] = B[j][l]), so both operands
// load 16 consecutive rows per instruction, and the operands of the next
// 16 values of k are loaded while the MFMAs of the current ones run.  C
// differs from A, B and D unless beta = 0.  Ends with a barrier.
__device__ void gmm_sym(double* C, int ldc, const double* A, int lda, const double* B, int ldb, int n, double alpha,
                        double beta, const double* D, int ldd) {
  constexpr int KC = 16, NL = KC / 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int nw = SNW;  // called by STHR-thread kernels only
  const int l16 = lane & 15, kq = lane >> 4;
  const int tn = wdiv(n, 16);
  const int ntiles = tn * (tn + 1) / 2;
  const int nch = wdiv(n, KC);
  for (int tile = wave; tile < ntiles; tile += nw) {
    int tj = 0, ti = tile;
    while (ti > tj) {
      ti -= tj + 1;
      ++tj;
    }
    const int i0 = 16 * ti, j0 = 16 * tj;
    const int i = i0 + l16, j = j0 + l16;
    const double* pa = A + (i < n ? i : 0);
    const double* pb = B + (j < n ? j : 0);
    auto load = [&](int c, double (&av)[NL], double (&bv)[NL]) {
#pragma unroll
      for (int u = 0; u < NL; ++u) {
        const int l = c * KC + 4 * u + kq;
        const int lc = l < n ? l : 0;
        const double a_ = pa[(int64_t)lc * lda], b_ = pb[(int64_t)lc * ldb];
        av[u] = (i < n && l < n) ? a_ : 0.0;
        bv[u] = (j < n && l < n) ? b_ : 0.0;
      }
    };
    dbl4 e = zero4(), o = zero4();
    double a0[NL], b0[NL], a1[NL], b1[NL];
    load(0, a0, b0);
    for (int c = 0; c < nch; c += 2) {
      if (c + 1 < nch) load(c + 1, a1, b1);
#pragma unroll
      for (int u = 0; u < NL; u += 2) {
        e = mfma64(a0[u], b0[u], e);
        o = mfma64(a0[u + 1], b0[u + 1], o);
      }
      if (c + 1 >= nch) break;
      if (c + 2 < nch) load(c + 2, a0, b0);
#pragma unroll
      for (int u = 0; u < NL; u += 2) {
        e = mfma64(a1[u], b1[u], e);
        o = mfma64(a1[u + 1], b1[u + 1], o);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ci = i0 + 4 * v + kq, cj = j0 + l16;
      if (ci < n && cj < n && (ti != tj || ci <= cj)) {
        const double acc = e[v] + o[v];
        const double val = beta == 0.0 ? alpha * acc : fma(alpha, acc, beta * D[ci + (int64_t)cj * ldd]);
        C[ci + (int64_t)cj * ldc] = val;
        C[cj + (int64_t)ci * ldc] = val;
      }
    }
  }
  __syncthreads();
}


// |C| = sign(C) C for a symmetric t x t matrix C (ld ld) into out, by the
// scaled Newton-Schulz iteration of Chen and Chow (2014) on X0 = C / |C|_F:
//   X <- a X (3 I - a^2 X^2) / 2,  a = sqrt(3 / (1 + l + l^2)),
// which maps eigenvalues in [l, 1] into [l', 1], l' = a l (3 - a^2 l^2) / 2,
// started from l = 1e-4 / sqrt(t), then the unscaled iteration
// X <- X (3 I - X^2) / 2 until an update moves X by at most 1e-14
// (Frobenius, at most 48 steps).  Eigenvalues below the scaled phase's bound
// keep their sign; exactly zero ones stay zero.  X, Y and W are t x t work
// buffers (ld ld).  Then C+ = (C + |C|) / 2 = P diag(max(lambda, 0)) P^T and
// C- = (C - |C|) / 2 without the eigenvectors.  STHR threads.
__device__ void ns_abs(const double* C, double* X, double* Y, double* W, double* out, int t, int ld, double* red) {
  double part = 0.0;
  for (int idx = threadIdx.x; idx < t * t; idx += STHR) {
    const double c = C[(idx % t) + (int64_t)(idx / t) * ld];
    part = fma(c, c, part);
  }
  const double fro = sqrt(s_sum(part, red));
  if (!(fro > 0.0)) {
    for (int idx = threadIdx.x; idx < t * t; idx += STHR) out[(idx % t) + (int64_t)(idx / t) * ld] = 0.0;
    __syncthreads();
    return;
  }
  const double ifro = 1.0 / fro;
  for (int idx = threadIdx.x; idx < t * t; idx += STHR) {
    const int o = (idx % t) + (idx / t) * ld;
    X[o] = C[o] * ifro;
  }
  __syncthreads();
  double l = 1e-4 / sqrt((double)t);
  for (int it = 0; it < 64 && 1.0 - l > 1e-15; ++it) {
    const double a2 = 3.0 / (1.0 + l + l * l), a = sqrt(a2);
    const double c1 = 1.5 * a, c3 = -0.5 * a * a2;
    gmm_sym(Y, ld, X, ld, X, ld, t, 1.0, 0.0, Y, ld);   // X^2
    gmm_sym(W, ld, X, ld, Y, ld, t, c3, c1, X, ld);     // c1 X + c3 X^3
    double* sw = X;
    X = W;
    W = sw;
    l = l * (c1 + c3 * l * l);
  }
  for (int it = 0; it < 48; ++it) {
    gmm_sym(Y, ld, X, ld, X, ld, t, 1.0, 0.0, Y, ld);
    gmm_sym(W, ld, X, ld, Y, ld, t, -0.5, 1.5, X, ld);
    double ch = 0.0;
    for (int idx = threadIdx.x; idx < t * t; idx += STHR) {
      const int o = (idx % t) + (idx / t) * ld;
      const double dl = W[o] - X[o];
      ch = fma(dl, dl, ch);
    }
    const double ch2 = s_sum(ch, red);
    double* sw = X;
    X = W;
    W = sw;
    if (ch2 <= 1e-28) break;
  }
  gmm_sym(out, ld, X, ld, C, ld, t, 1.0, 0.0, out, ld);  // sign(C) C
}

// Right-looking Cholesky G = L L^T of the n x n matrix in LDS (ld WLD,
// n <= 128), L written over its lower triangle; the matrix being reduced
// is held in registers, so each column costs two barriers and no LDS
// traffic beyond the column itself.  dep[k] = 1 marks a pivot at most
// 1e-20 of its initial diagonal d0[k] (or not finite): its column is set to
// the unit vector, so the factorisation goes on.  Returns the smallest ratio
// pivot / d0 met (for the unshifted first try).  The strict upper triangle
// is zeroed on exit.  col: n doubles of LDS scratch.  STHR threads.
__device__ double lds_chol(const Dev& d, double* L, int n, const double* d0, int* dep, double* red, double* col) {
  // the active matrix in registers: thread t < CTHR, (ri, ci) = (t % 16,
  // t / 16), holds rows 8 ri .. 8 ri + 7 and columns 4 ci .. 4 ci + 3 of the
  // full square (both triangles get the same updates), so the holders of a
  // column are 16 lanes of one wavefront; each step's column goes through
  // LDS (col) and its scaled values into L.  The other wavefronts only keep
  // the barriers: the per-step work that every wavefront repeats (the
  // pivot's square root and reciprocal, the column reads) is issued by half
  // as many.
  constexpr int CTHR = 512;
  static_assert(8 * 16 >= WCAP_T && 4 * (CTHR / 16) >= WCAP_T && STHR >= CTHR, "register tiles of the Gram");
  double& minratio = red[SNW];
  const bool act = threadIdx.x < CTHR;
  const int ri = threadIdx.x & 15, ci = (threadIdx.x >> 4) & (CTHR / 16 - 1);
  double g[8][4];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = 8 * ri + a, j = 4 * ci + b;
      g[a][b] = (act && i < n && j < n) ? L[i + j * WLD] : 0.0;
    }
  if (threadIdx.x == 0) minratio = 1e300;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    // the holders of column k publish it
    if (act && ci == (k >> 2)) {
      const int cc = k & 3;
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        double v = 0.0;
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if (b == cc) v = g[a][b];
        if (8 * ri + a < n) col[8 * ri + a] = v;
      }
    }
    __syncthreads();
    if (act) {
      const double pv = col[k];
      const bool isdep = !isfinite(pv) || !(pv > 1e-20 * d0[k]);
      const double lkk = isdep ? 1.0 : sqrt(pv);
      const double il = 1.0 / lkk;
      if (threadIdx.x == 0) {
        dep[k] = isdep ? 1 : 0;
        minratio = fmin(minratio, isdep ? 0.0 : pv / d0[k]);
        L[k + k * WLD] = lkk;
        if (!isfinite(pv)) atomicOr(d.flags, FLAG_NONFINITE);
      }
      for (int i = k + 1 + (int)threadIdx.x; i < n; i += CTHR) L[i + k * WLD] = isdep ? 0.0 : col[i] * il;
      double li[8], lj[4];
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int i = 8 * ri + a;
        li[a] = (i > k && i < n && !isdep) ? col[i] * il : 0.0;
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int j = 4 * ci + b;
        lj[b] = (j > k && j < n && !isdep) ? col[j] * il : 0.0;
      }
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) g[a][b] = fma(-li[a], lj[b], g[a][b]);
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < n * n; idx += STHR) {
    const int i = idx % n, j = idx / n;
    if (i < j) L[i + j * WLD] = 0.0;
  }
  __syncthreads();
  const double mr = minratio;
  __syncthreads();
  return mr;
}

// In-place inverse of the lower triangular L (n x n, LDS, ld WLD, unit
// vectors in dependent columns keep it regular), column by column from the
// last: X[j][j] = 1/L[j][j], X[i][j] = -X[j][j] sum_{j<l<=i} X[i][l] L[l][j].
// Each row's sum is split over 8 lanes and added with DPP (STHR threads).
__device__ void lds_tri_inv(double* L, int n, double* colj) {
  for (int j = n - 1; j >= 0; --j) {
    for (int i = threadIdx.x; i < n; i += STHR) colj[i] = L[i + j * WLD];
    __syncthreads();
    const double xjj = 1.0 / colj[j];
    const int grp = threadIdx.x >> 3, sub = threadIdx.x & 7;
    double val = 0.0;
    const int i = j + 1 + grp;
    if (i < n) {
      for (int l = j + 1 + sub; l <= i; l += 8) val = fma(L[i + l * WLD], colj[l], val);
    }
    val = group_sum_dpp<8>(val);
    __syncthreads();
    if (i < n && sub == 0) L[i + j * WLD] = -xjj * val;
    if (threadIdx.x == 0) L[j + j * WLD] = xjj;
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// One-sided Jacobi with the columns in registers ("group ring").  The SVD
// kernels run JTHR threads; lane l of a wavefront belongs to group l % 4, so
// each wavefront holds four groups of 16 lanes, and group gi = 4 wave + l % 4
// holds the pair slots p = gi PPG + k (k < PPG): a top and a bottom column,
// row l / 4 + 16 i in register i of lane l, with ACC the matching columns
// of the accumulated rotation J, and the squared norms of both columns (the
// same value in every lane of the group).  A pair's inner product is summed
// over its 16 lanes by partner exchanges (DPP row rotations by 8 and 4, then
// swaps of rows and of wavefront halves), each of which adds the same two
// values on both sides, so every lane of the group gets the same bits and
// forms the same rotation: four pairs share each instruction and no value
// has to be read back from a single lane.
//
// After each round the columns move by the caterpillar rule
//   top'[0] = top[0], top'[1] = bot[0], top'[p] = top[p-1] (p >= 2),
//   bot'[p] = bot[p+1] (p <= P-2), bot'[P-1] = top[P-1],
// which meets every pair once in n2 - 1 rounds.  Inside a group the moves
// are renamings: in phase ph of the round counter (mod PPG) logical top k is
// register (k - ph) mod PPG and logical bottom k is register (k + ph) mod
// PPG, so only the outgoing top of the last slot and the outgoing bottom of
// the first slot of each group move: to the neighbouring group of the same
// wavefront by a DPP rotation inside each quad of lanes, across wavefronts
// through a double-buffered LDS area (one barrier per round).  Slots p >= P
// are inactive: they never rotate, and what drifts into them never flows
// back.  The squared norms are updated with each rotation (|x'|^2 = c^2 |x|^2
// - 2 c s x.y + s^2 |y|^2, and likewise) and recomputed exactly at the start
// of every sweep.
// ----------------------------------------------------------------------------
constexpr int JTHR = 512;          // threads of the SVD kernels
constexpr int JNW = JTHR / 64;
constexpr int JNG = 4 * JNW;       // lane groups of 16

template <int PPG, int RPL, bool ACC, int JRPL>
struct GRing {
  static constexpr int JR = ACC ? JRPL : 1;
  static constexpr int CW = RPL + (ACC ? JRPL : 0) + 1;  // values per lane of one moving column
  double t[RPL][PPG], b[RPL][PPG];
  double jt[JR][PPG], jb[JR][PPG];
  double nt[PPG], nb[PPG];
};

// LDS doubles of the wavefront-boundary exchange: [buffer][direction][wave][CW][16]
template <int CW>
constexpr int gring_lds_doubles() { return 2 * 2 * JNW * CW * 16; }

// a double swapped between the two rows of each pair of rows (R = 16) or
// between the two halves of the wavefront (R = 32): returns both values, in
// the same order on both sides
template <int R>
__device__ __forceinline__ void lane_swap(double v, double& a, double& b) {
  union { double d; unsigned u[2]; } x, p, q;
  x.d = v;
  if (R == 16) {
    const auto lo = __builtin_amdgcn_permlane16_swap(x.u[0], x.u[0], false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(x.u[1], x.u[1], false, false);
    p.u[0] = lo[0]; q.u[0] = lo[1]; p.u[1] = hi[0]; q.u[1] = hi[1];
  } else {
    const auto lo = __builtin_amdgcn_permlane32_swap(x.u[0], x.u[0], false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(x.u[1], x.u[1], false, false);
    p.u[0] = lo[0]; q.u[0] = lo[1]; p.u[1] = hi[0]; q.u[1] = hi[1];
  }
  a = p.d;
  b = q.d;
}

// sum over the 16 lanes of a group (lanes of one residue mod 4), the same
// bits in every one of them
__device__ __forceinline__ double class_sum16(double v) {
  v += dpp_double<0x128>(v);  // row_ror:8, partner lane i + 8 in its row
  v += dpp_double<0x124>(v);  // row_ror:4 (the values repeat with period 8 now)
  double a, b;
  lane_swap<16>(v, a, b);
  v = a + b;
  lane_swap<32>(v, a, b);
  return a + b;
}

// the value of the previous / next group of the same quad (group 0 gets
// group 3's, group 3 gets group 0's)
__device__ __forceinline__ double from_prev_group(double v) { return dpp_double<0x93>(v); }  // quad_perm [3,0,1,2]
__device__ __forceinline__ double from_next_group(double v) { return dpp_double<0x39>(v); }  // quad_perm [1,2,3,0]

// a lane's place in the group ring
struct GPos {
  int l16, g, wave, gi;
  int P, gP, kP;        // active pair slots, group and slot of the last one
  bool special;         // the wavefront holds slot 0 or slot P - 1 (uniform)
  bool rdT, rdB;        // the lane takes its incoming top / bottom from LDS
};

// The moves of one row inside a wavefront (T[k] / B[k]: the row's values
// in the top / bottom registers k).  Lanes of groups 0 and 3 receive a value
// here that is replaced after the barrier.  The special form also applies
// the rules of the two ends of the ring: slot 0 keeps its top and takes its
// bottom as top'[1], and the last active slot P - 1 takes its top as its
// new bottom.
template <int PPG, int PH>
__device__ __forceinline__ void gx_plain(double (&T)[PPG], double (&B)[PPG], const GPos& x) {
  constexpr int OTP = (2 * PPG - 1 - PH) % PPG;  // logical top PPG-1
  constexpr int OBP = PH % PPG;                   // logical bottom 0
  T[OTP] = from_prev_group(T[OTP]);
  B[OBP] = from_next_group(B[OBP]);
}

template <int PPG, int PH>
__device__ __forceinline__ void gx_special(double (&T)[PPG], double (&B)[PPG], const GPos& x) {
  constexpr int OTP = (2 * PPG - 1 - PH) % PPG;
  constexpr int OBP = PH % PPG;
  constexpr int T0P = (PPG - PH) % PPG;           // logical top 0
  const double oldT = T[OTP], oldB = B[OBP], t0 = T[T0P];
  const double inT = from_prev_group(oldT), inB = from_next_group(oldB);
  const bool last = x.gi == x.gP;
#pragma unroll
  for (int kk = 0; kk + 1 < PPG; ++kk)
    if (last && x.kP == kk) B[(kk + PH + 1) % PPG] = T[(kk - PH + PPG) % PPG];
  B[OBP] = (last && x.kP == PPG - 1) ? oldT : inB;
  T[OTP] = x.gi == 0 ? t0 : inT;
  if (x.gi == 0) T[T0P] = oldB;
}

// One round in phase PH: rotate every active pair, then move the columns.
// Returns true if this lane rotated a pair.
template <int PH, int PPG, int RPL, bool ACC, int JRPL>
__device__ __forceinline__ bool gring_round(GRing<PPG, RPL, ACC, JRPL>& c, const GPos& x, double floor2, double tol2,
                                            bool move, double* xbuf, int buf) {
  using GR = GRing<PPG, RPL, ACC, JRPL>;
  bool rot = false;
  if (__builtin_amdgcn_readfirstlane(x.wave) * 4 * PPG < x.P) {  // a wavefront with active slots
    double ga[PPG];
#pragma unroll
    for (int k = 0; k < PPG; ++k) {
      const int pt = (k - PH + PPG) % PPG, pb = (k + PH) % PPG;
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < RPL; ++i) s = fma(c.t[i][pt], c.b[i][pb], s);
      ga[k] = class_sum16(s);
    }
#pragma unroll
    for (int k = 0; k < PPG; ++k) {
      const int pt = (k - PH + PPG) % PPG, pb = (k + PH) % PPG;
      const double al = c.nt[pt], be = c.nb[pb], g = ga[k];
      const bool act = x.gi * PPG + k < x.P;
      const bool dorot = act && g != 0.0 && al > floor2 && be > floor2 && g * g > tol2 * al * be;
      // every lane applies a rotation, the identity (c = 1, s = 0: exact)
      // where the pair is left alone, so no branch splits the groups
      double cs, sn;
      jacobi_rotation(al, be, g, cs, sn);
      cs = dorot ? cs : 1.0;
      sn = dorot ? sn : 0.0;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const double u = c.t[i][pt], v = c.b[i][pb];
        c.t[i][pt] = cs * u - sn * v;
        c.b[i][pb] = fma(sn, u, cs * v);
      }
      if (ACC) {
#pragma unroll
        for (int i = 0; i < GR::JR; ++i) {
          const double u = c.jt[i][pt], v = c.jb[i][pb];
          c.jt[i][pt] = cs * u - sn * v;
          c.jb[i][pb] = fma(sn, u, cs * v);
        }
      }
      const double cg = 2.0 * cs * sn * g;
      c.nt[pt] = fma(cs * cs, al, fma(sn * sn, be, -cg));
      c.nb[pb] = fma(sn * sn, al, fma(cs * cs, be, cg));
      rot = rot || dorot;
    }
  }
  if (!move) return rot;
  constexpr int CW = GR::CW;
  constexpr int OTP = (2 * PPG - 1 - PH) % PPG, OBP = PH % PPG;
  double* ob = xbuf + buf * (2 * JNW * CW * 16);
  // outgoing columns of the wavefront's end groups, [buffer][direction]
  // [wave][value][16]: the top of group 3 (direction 0), the bottom of
  // group 0 (direction 1); one store per value and lane, the value selected
  // (a store from either column would take the columns out of registers)
  if (x.g == 0 || x.g == 3) {
    const bool up = x.g == 3;
    double* o = ob + ((up ? 0 : JNW) + x.wave) * CW * 16 + x.l16;
#pragma unroll
    for (int i = 0; i < RPL; ++i) o[i * 16] = up ? c.t[i][OTP] : c.b[i][OBP];
    if (ACC) {
#pragma unroll
      for (int i = 0; i < GR::JR; ++i) o[(RPL + i) * 16] = up ? c.jt[i][OTP] : c.jb[i][OBP];
    }
    o[(CW - 1) * 16] = up ? c.nt[OTP] : c.nb[OBP];
  }
  if (x.special) {
#pragma unroll
    for (int i = 0; i < RPL; ++i) gx_special<PPG, PH>(c.t[i], c.b[i], x);
    if (ACC) {
#pragma unroll
      for (int i = 0; i < GR::JR; ++i) gx_special<PPG, PH>(c.jt[i], c.jb[i], x);
    }
    gx_special<PPG, PH>(c.nt, c.nb, x);
  } else {
#pragma unroll
    for (int i = 0; i < RPL; ++i) gx_plain<PPG, PH>(c.t[i], c.b[i], x);
    if (ACC) {
#pragma unroll
      for (int i = 0; i < GR::JR; ++i) gx_plain<PPG, PH>(c.jt[i], c.jb[i], x);
    }
    gx_plain<PPG, PH>(c.nt, c.nb, x);
  }
  __syncthreads();
  // incoming columns across wavefronts: group 0 takes the previous
  // wavefront's top, group 3 the next wavefront's bottom
  if (x.rdT) {
    const double* q = ob + (x.wave - 1) * CW * 16 + x.l16;
#pragma unroll
    for (int i = 0; i < RPL; ++i) c.t[i][OTP] = q[i * 16];
    if (ACC) {
#pragma unroll
      for (int i = 0; i < GR::JR; ++i) c.jt[i][OTP] = q[(RPL + i) * 16];
    }
    c.nt[OTP] = q[(CW - 1) * 16];
  }
  if (x.rdB) {
    const double* q = ob + (JNW + x.wave + 1) * CW * 16 + x.l16;
#pragma unroll
    for (int i = 0; i < RPL; ++i) c.b[i][OBP] = q[i * 16];
    if (ACC) {
#pragma unroll
      for (int i = 0; i < GR::JR; ++i) c.jb[i][OBP] = q[(RPL + i) * 16];
    }
    c.nb[OBP] = q[(CW - 1) * 16];
  }
  return rot;
}

// registers of phase ph back to phase 0 (logical slot k in register k)
template <int PPG>
__device__ __forceinline__ void gring_unphase(double (&T)[PPG], double (&B)[PPG], int ph) {
  double t2[PPG], b2[PPG];
#pragma unroll
  for (int q = 1; q < PPG; ++q) {
    if (ph != q) continue;
#pragma unroll
    for (int k = 0; k < PPG; ++k) {
      t2[k] = T[(k - q + PPG) % PPG];
      b2[k] = B[(k + q) % PPG];
    }
#pragma unroll
    for (int k = 0; k < PPG; ++k) {
      T[k] = t2[k];
      B[k] = b2[k];
    }
  }
}

// exact squared norms of every register's columns
template <int PPG, int RPL, bool ACC, int JRPL>
__device__ __forceinline__ void gring_norms(GRing<PPG, RPL, ACC, JRPL>& c) {
#pragma unroll
  for (int k = 0; k < PPG; ++k) {
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      a = fma(c.t[i][k], c.t[i][k], a);
      b = fma(c.b[i][k], c.b[i][k], b);
    }
    c.nt[k] = class_sum16(a);
    c.nb[k] = class_sum16(b);
  }
}

// sweep bookkeeping of the group ring
struct GSweep {
  int rr;         // rounds done in the current sweep
  int sweeps;     // current sweep (1-based)
  int buf;        // exchange buffer of the next round
  bool rot;       // this lane rotated a pair in the current sweep
  bool converged;
};

// One round in phase PH and, after the last round of a sweep, the sweep's
// end: the block stops when no wavefront rotated (converged) or after
// max_sweeps, else the next sweep starts from exact norms.  Returns true
// when the block stops.
template <int PH, int PPG, int RPL, bool ACC, int JRPL>
__device__ __forceinline__ bool gring_step(GRing<PPG, RPL, ACC, JRPL>& c, const GPos& x, double floor2, double tol2,
                                           bool move, double* xbuf, int* rotflag, int n2, int max_sweeps,
                                           GSweep& w) {
  const bool r = gring_round<PH>(c, x, floor2, tol2, move, xbuf, w.buf);
  w.rot = w.rot || r;
  w.buf ^= 1;
  if (++w.rr < n2 - 1) return false;
  // after n2 - 1 rounds every column is back in its starting slot
  w.rr = 0;
  const bool any = __any(w.rot ? 1 : 0);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) rotflag[x.wave] = any ? 1 : 0;
  __syncthreads();
  int anyb = 0;
  for (int q = 0; q < JNW; ++q) anyb |= rotflag[q];
  __syncthreads();
  if (!anyb) {
    w.converged = true;
    return true;
  }
  if (w.sweeps == max_sweeps) return true;
  ++w.sweeps;
  w.rot = false;
  gring_norms(c);
  return false;
}

// Runs the sweeps on the n columns held in c (rows <= 16 RPL each); on
// return logical slot k is in register k again.  Returns the sweeps done
// (negative if not converged within max_sweeps).
template <int PPG, int RPL, bool ACC, int JRPL>
__device__ __forceinline__ int gring_jacobi(const Dev& d, GRing<PPG, RPL, ACC, JRPL>& c, int n, double tol, double floor_rel,
                            int max_sweeps, double* xbuf, double* red, int* rotflag) {
  static_assert(PPG >= 2, "two pair slots per group at least");
  using GR = GRing<PPG, RPL, ACC, JRPL>;
  GPos x;
  const int lane = threadIdx.x & 63;
  x.l16 = lane >> 2;
  x.g = lane & 3;
  x.wave = threadIdx.x >> 6;
  x.gi = 4 * x.wave + x.g;
  const int n2 = n + (n & 1);
  x.P = n2 / 2;
  x.gP = x.P > 0 ? (x.P - 1) / PPG : 0;
  x.kP = x.P > 0 ? (x.P - 1) % PPG : 0;
  const int uw = __builtin_amdgcn_readfirstlane(x.wave);
  x.special = uw == 0 || uw == x.gP / 4;
  x.rdT = x.g == 0 && x.gi != 0;
  x.rdB = x.g == 3 && x.wave + 1 < JNW && !(x.gi == x.gP && x.kP == PPG - 1);
  double part = 0.0;
#pragma unroll
  for (int i = 0; i < RPL; ++i)
#pragma unroll
    for (int k = 0; k < PPG; ++k) part = fma(c.t[i][k], c.t[i][k], fma(c.b[i][k], c.b[i][k], part));
  const double floor2 = floor_rel * floor_rel * s_sum(part, red);
  const double tol2 = tol * tol;
  if (n2 <= 1) return 0;
  GSweep w{0, 1, 0, false, false};
  gring_norms(c);
  int ph = 0;
  if (x.P == 1) {
    // a single pair: nothing moves
    while (!gring_step<0>(c, x, floor2, tol2, false, xbuf, rotflag, n2, max_sweeps, w)) {
    }
  } else {
    // the round loop unrolled over the phases, so that every register keeps
    // its role from one round to the next
    for (;;) {
      if (gring_step<0>(c, x, floor2, tol2, true, xbuf, rotflag, n2, max_sweeps, w)) {
        ph = 1 % PPG;
        break;
      }
      if (gring_step<1 % PPG>(c, x, floor2, tol2, true, xbuf, rotflag, n2, max_sweeps, w)) {
        ph = 2 % PPG;
        break;
      }
      if constexpr (PPG > 2) {
        if (gring_step<2 % PPG>(c, x, floor2, tol2, true, xbuf, rotflag, n2, max_sweeps, w)) {
          ph = 3 % PPG;
          break;
        }
      }
    }
  }
  const bool converged = w.converged;
  const int sweeps = w.sweeps;
#pragma unroll
  for (int i = 0; i < RPL; ++i) gring_unphase<PPG>(c.t[i], c.b[i], ph);
  if (ACC) {
#pragma unroll
    for (int i = 0; i < GR::JR; ++i) gring_unphase<PPG>(c.jt[i], c.jb[i], ph);
  }
  gring_unphase<PPG>(c.nt, c.nb, ph);
  if (!converged && threadIdx.x == 0) atomicOr(d.flags, FLAG_JACOBI_NOCONV);
  return converged ? sweeps : -sweeps;
}

// rank of the value of column c among n values (descending, ties by index)
__device__ __forceinline__ int desc_rank(const double* v, int n, int c) {
  const double x = v[c];
  int r = 0;
  for (int k = 0; k < n; ++k) r += (v[k] > x || (v[k] == x && k < c)) ? 1 : 0;
  return r;
}

// ============================================================================
// small kernels
// ============================================================================

// LDS scratch of a wide small kernel, declared once per kernel (arrays
// declared inside the templated bodies would be allocated once per
// instantiation).
struct SmallScratch {
  double red[SNW + 2];
  int rotflag[SNW];
  double v0[WCAP_A], v1[WCAP_A], v2[WCAP_A], v3[WCAP_A], v4[WCAP_A];
  int i0[WCAP_A], i1[WCAP_A];
  int ival[4];
};

// One pass of (shifted) Cholesky QR for the wide plan, n <= 128: sum of the
// partial Grams, the factor G = R^T R (tried unshifted first; when a pivot
// keeps less than 1e-12 of its diagonal the Gram is summed again with the
// shift 11 (rows n + n (n+1)) u tr(G) of Fukaya et al. and factored again),
//   Rinv slot: bscale R^{-1},  fill slot: dependent columns,
//   Racc slot: R (acc_mode 1) or R Racc (acc_mode 2), rows of dependent
//              columns zeroed.
__global__ __launch_bounds__(STHR) void sw_chol(Dev d, int axis, int sd0, int ndim, int rows, int ngp, int acc_mode,
                                               double bscale, int oRinv, int oRacc, int ld, int near, int skip_mode) {
  const int s = sd0 + blockIdx.x;
  const int n = dim_of(d, s, axis, ndim);
  double* sm = small_of(d, s);
  extern __shared__ double L[];  // n x n, ld WLD
  __shared__ SmallScratch sc;
  double* d0 = sc.v0;
  int* dep = sc.i0;
  if (n <= 0) return;
  // a pass after one that took the near-identity factor is skipped: that
  // output is orthonormal to rounding, R = I (Racc unchanged), and the Gram
  // and the product of this pass are skipped with it
  if (skip_mode == 2 && sm[d.oSkip] != 0.0) return;
  if (near) {
    // A Gram within 1e-3 (Frobenius) of the identity (a pass over an input
    // that is already orthonormal up to rounding) takes the symmetric factor
    // from the binomial series in E = G - I:
    //   R    = I + E/2 - E^2/8 + E^3/16 - 5 E^4/128,
    //   R^-1 = I - E/2 + 3 E^2/8 - 5 E^3/16 + 35 E^4/128,
    // cut after E^2 when |E|^2 <= 1e-10 (remainder 0.3 |E|^3 <= 3e-16) and
    // after E^4 otherwise (remainder 0.25 |E|^5 <= 2.5e-16); any R with
    // G = R^T R gives an orthonormal Q = X R^-1.
    const int T = d.T;
    double* E = sm + d.oW2;
    double* E2 = sm + d.oW3;
    double* E3 = sm + d.oW4;
    double* E4 = sm + d.oW5;
    s_sum_partials(d, s, ngp, 0, n, n, n, E, T, 1.0);
    __syncthreads();
    double part = 0.0;
    for (int idx = threadIdx.x; idx < n * n; idx += STHR) {
      const int i = idx % n, j = idx / n;
      // symmetrise, subtract the identity
      const double e = 0.5 * (E[i + j * T] + E[j + i * T]) - (i == j ? 1.0 : 0.0);
      L[i + j * WLD] = e;
      part = fma(e, e, part);
    }
    const double fro2 = s_sum(part, sc.red);
    if (fro2 <= 1e-6) {
      for (int idx = threadIdx.x; idx < n * n; idx += STHR) {
        const int i = idx % n, j = idx / n;
        E[i + j * T] = L[i + j * WLD];
      }
      __syncthreads();
      const bool o4 = fro2 > 1e-10;
      gmm_sym(E2, T, E, T, E, T, n, 1.0, 0.0, E2, T);
      if (o4) {
        gmm_sym(E3, T, E, T, E2, T, n, 1.0, 0.0, E3, T);
        gmm_sym(E4, T, E2, T, E2, T, n, 1.0, 0.0, E4, T);
      }
      for (int idx = threadIdx.x; idx < n * n; idx += STHR) {
        const int i = idx % n, j = idx / n;
        const int o = i + j * T;
        const double id = i == j ? 1.0 : 0.0, e = E[o], e2 = E2[o];
        double r = id + 0.5 * e - 0.125 * e2, ri = id - 0.5 * e + 0.375 * e2;
        if (o4) {
          r += 0.0625 * E3[o] - 0.0390625 * E4[o];
          ri += -0.3125 * E3[o] + 0.2734375 * E4[o];
        }
        L[i + j * WLD] = r;
        sm[oRinv + i + j * ld] = bscale * ri;
      }
      for (int j = threadIdx.x; j < n; j += STHR) sm[d.oFill + j] = 0.0;
      __syncthreads();
      if (acc_mode == 1) {
        for (int idx = threadIdx.x; idx < n * n; idx += STHR) {
          const int i = idx % n, j = idx / n;
          sm[oRacc + i + j * ld] = L[i + j * WLD];
        }
      } else if (acc_mode == 2) {
        double* Wt = sm + d.oW1;
        gmm(Wt, T, L, WLD, false, sm + oRacc, ld, false, n, n, n, 1.0, 0.0);
        for (int idx = threadIdx.x; idx < n * n; idx += STHR) {
          const int i = idx % n, j = idx / n;
          sm[oRacc + i + j * ld] = Wt[i + j * T];
        }
      }
      if (skip_mode == 1 && threadIdx.x == 0) sm[d.oSkip] = 1.0;
      return;
    }
  }
  if (skip_mode == 1 && threadIdx.x == 0) sm[d.oSkip] = 0.0;
  bool shifted = false;
  for (int attempt = 0; attempt < 2; ++attempt) {
    s_sum_partials(d, s, ngp, 0, n, n, n, L, WLD, 1.0);
    __syncthreads();
    if (shifted) {
      double part = 0.0;
      for (int i = threadIdx.x; i < n; i += STHR) part += L[i * (WLD + 1)];
      const double tr = s_sum(part, sc.red);
      const double sh = 11.0 * ((double)rows * n + (double)n * (n + 1)) * U_ROUND * tr;
      for (int i = threadIdx.x; i < n; i += STHR) L[i * (WLD + 1)] += sh;
      __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += STHR) d0[i] = L[i * (WLD + 1)];
    __syncthreads();
    const double mr = lds_chol(d, L, n, d0, dep, sc.red, sc.v1);
    if (shifted || mr >= 1e-12) break;
    shifted = true;
  }
  // Racc update before L is inverted: R = L^T
  double* Wt = sm + d.oW1;  // T x T scratch
  if (acc_mode == 1) {
    for (int idx = threadIdx.x; idx < n * n; idx += STHR) {
      const int i = idx % n, j = idx / n;
      sm[oRacc + i + j * ld] = (dep[i] || i > j) ? 0.0 : L[j + i * WLD];
    }
  } else if (acc_mode == 2) {
    gmm(Wt, d.T, L, WLD, true, sm + oRacc, ld, false, n, n, n, 1.0, 0.0);
    for (int idx = threadIdx.x; idx < n * n; idx += STHR) {
      const int i = idx % n, j = idx / n;
      sm[oRacc + i + j * ld] = dep[i] ? 0.0 : Wt[i + j * d.T];
    }
  }
  __syncthreads();
  lds_tri_inv(L, n, sc.v1);
  // R^{-1} = (L^{-1})^T
  for (int idx = threadIdx.x; idx < n * n; idx += STHR) {
    const int i = idx % n, j = idx / n;
    sm[oRinv + i + j * ld] = i <= j ? bscale * L[j + i * WLD] : 0.0;
  }
  for (int j = threadIdx.x; j < n; j += STHR) sm[d.oFill + j] = dep[j] ? 1.0 : 0.0;
}

// Augmentation SVD (Algorithm 4, steps 2-4) for widths m0 <= 192: the Gram
// G = A^T A of A = sqrt(w) L0 is factored by a diagonally pivoted Cholesky
// (packed lower triangle in LDS) that stops when the largest remaining pivot
// is at most 1e-20 of the largest initial diagonal; the columns of the
// factor L (G[perm, perm] = L L^T, rows in the original order) are then
// orthogonalised by the group ring Jacobi, L J = B, so that A B Sigma^-2 has
// orthonormal columns: the left singular vectors of A, with sigma the
// column norms of B.  Then the rank rule of step 3 and the coefficients of
// sqrt(w) V-hat = A B[:, :t] Sigma^-2.  Singular values come from the Gram:
// they are accurate to about u sigma_1^2 / sigma, which resolves the
// absolute tolerances of the adaptive mode.
template <int PPG, int RPL>
__device__ __forceinline__ void aug_svd_body(const Dev& d, int s, int axis, int m0, double* lds, SmallScratch& sc) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane >> 2, gi = 4 * wave + (lane & 3);
  double* sm = small_of(d, s);
  const int r = d.rank[s];
  double* Gp = lds;            // packed lower triangle, m0 (m0 + 1) / 2
  double* dg = sc.v0;          // current diagonal
  double* d0s = sc.v1;
  int* estep = sc.i0;          // elimination step of each column (NOT_ELIM: never)
  double* lcol = sc.v2;        // the step's factor column, 0 outside the remaining rows
  double* sigs = sc.v3;
  double* sorted = sc.v4;
  int* rk = sc.i1;
  constexpr int NOT_ELIM = 1 << 20;
  auto pk = [](int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; };
  // Gram from the partials (symmetric, ld m0), lower triangle packed:
  // columns j over the wavefronts, rows i >= j over the lanes
  {
    const double* gp = gpart_of(d, s);
    const int ngp = d.xgM;  // the Gram of A is reduced into at most 8 partials
    constexpr int UI = 2;
    for (int j = wave; j < m0; j += JNW)
      for (int i0 = j + lane; i0 < m0; i0 += 64 * UI) {
        int64_t src[UI];
#pragma unroll
        for (int u = 0; u < UI; ++u) {
          const int i = i0 + 64 * u;
          src[u] = i < m0 ? i + (int64_t)j * m0 : 0;
        }
        double acc[UI];
        sum_partials_multi<UI>(gp, d.gpTile, ngp, src, acc);
#pragma unroll
        for (int u = 0; u < UI; ++u) {
          const int i = i0 + 64 * u;
          if (i < m0) Gp[i * (i + 1) / 2 + j] = acc[u];
        }
      }
    __syncthreads();
    for (int i = threadIdx.x; i < m0; i += JTHR) {
      dg[i] = Gp[i * (i + 1) / 2 + i];
      d0s[i] = dg[i];
      estep[i] = NOT_ELIM;
    }
    __syncthreads();
  }
  double dmax = 0.0;
  for (int i = threadIdx.x; i < m0; i += JTHR) dmax = fmax(dmax, d0s[i]);
  dmax = s_max(dmax, sc.red);
  // the active Gram in registers: thread (ri, ci) = (tid / 32, tid % 32)
  // holds rows [12 ri, 12 ri + 12) and columns [6 ci, 6 ci + 6) of the full
  // square (both triangles get the same updates, so it stays symmetric);
  // the packed triangle in LDS then receives the factor columns
  constexpr int GR_ = 12, GC_ = 6;
  static_assert(GR_ * (JTHR / 32) >= WCAP_A && GC_ * 32 >= WCAP_A, "register tiles of the Gram");
  const int ri = threadIdx.x >> 5, ci = threadIdx.x & 31;
  double gt[GR_][GC_];
#pragma unroll
  for (int a = 0; a < GR_; ++a)
#pragma unroll
    for (int b = 0; b < GC_; ++b) {
      const int i = GR_ * ri + a, j = GC_ * ci + b;
      gt[a][b] = (i < m0 && j < m0) ? Gp[pk(i, j)] : 0.0;
    }
  __syncthreads();
  // pivoted right-looking Cholesky: pivot = the largest remaining diagonal,
  // the smallest index among equal ones (every wavefront finds it itself)
  for (int k = 0; k < m0; ++k) {
    double key = 0.0;
    for (int i = lane; i < m0; i += 64)
      if (estep[i] > k) key = fmax(key, dg[i]);
    const double best = wave_max(key);
    int p = m0;
    for (int q = 0; q * 64 < m0; ++q) {
      const int i = lane + 64 * q;
      const unsigned long long m = __ballot(i < m0 && estep[i] > k && dg[i] == best);
      if (m) {
        p = 64 * q + __builtin_ctzll(m);
        break;
      }
    }
    if (p >= m0 || !(best > 1e-20 * dmax) || !isfinite(best)) break;  // the rest is numerically dependent
    const double lpp = sqrt(best), il = 1.0 / lpp;
    // the step's factor column from the holders of Gram column p
    if (ci == p / GC_) {
      const int cc = p - GC_ * ci;
#pragma unroll
      for (int a = 0; a < GR_; ++a) {
        const int i = GR_ * ri + a;
        double v = 0.0;
#pragma unroll
        for (int b = 0; b < GC_; ++b)
          if (b == cc) v = gt[a][b];
        if (i < m0) lcol[i] = (i != p && estep[i] > k) ? v * il : 0.0;
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < m0; i += JTHR) {
      if (i != p && estep[i] > k) {   // the remaining rows (the rest of the column holds earlier factors)
        const double l = lcol[i];
        Gp[pk(i, p)] = l;
        dg[i] = fma(-l, l, dg[i]);
      }
    }
    if (threadIdx.x == 0) {
      Gp[pk(p, p)] = lpp;
      estep[p] = k;
    }
    double li[GR_], lj[GC_];
#pragma unroll
    for (int a = 0; a < GR_; ++a) li[a] = GR_ * ri + a < m0 ? lcol[GR_ * ri + a] : 0.0;
#pragma unroll
    for (int b = 0; b < GC_; ++b) lj[b] = GC_ * ci + b < m0 ? lcol[GC_ * ci + b] : 0.0;
#pragma unroll
    for (int a = 0; a < GR_; ++a)
#pragma unroll
      for (int b = 0; b < GC_; ++b) gt[a][b] = fma(-li[a], lj[b], gt[a][b]);
    __syncthreads();
  }
  // columns of the factor into the ring registers: column c (original
  // index) holds L(:, estep[c]), nonzero in rows eliminated at or after it
  GRing<PPG, RPL, false, 1> c;
#pragma unroll
  for (int i = 0; i < RPL; ++i)
#pragma unroll
    for (int k = 0; k < PPG; ++k) {
      const int row = l16 + 16 * i;
      const int p = gi * PPG + k;
      const int ct = 2 * p, cb = 2 * p + 1;
      double vt = 0.0, vb = 0.0;
      if (row < m0 && ct < m0 && estep[ct] < NOT_ELIM) {
        if (row == ct) vt = Gp[pk(ct, ct)];
        else if (estep[row] > estep[ct]) vt = Gp[pk(row, ct)];
      }
      if (row < m0 && cb < m0 && estep[cb] < NOT_ELIM) {
        if (row == cb) vb = Gp[pk(cb, cb)];
        else if (estep[row] > estep[cb]) vb = Gp[pk(row, cb)];
      }
      c.t[i][k] = vt;
      c.b[i][k] = vb;
    }
#pragma unroll
  for (int k = 0; k < PPG; ++k) c.nt[k] = c.nb[k] = 0.0;
  __syncthreads();  // LDS now free for the exchange buffers
  gring_jacobi<PPG, RPL, false, 1>(d, c, m0, 1e-14, 1e-15, 40, lds, sc.red, sc.rotflag);
  // singular values: column norms
#pragma unroll
  for (int k = 0; k < PPG; ++k) {
    double nt = 0.0, nb = 0.0;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      nt = fma(c.t[i][k], c.t[i][k], nt);
      nb = fma(c.b[i][k], c.b[i][k], nb);
    }
    nt = class_sum16(nt);
    nb = class_sum16(nb);
    const int p = gi * PPG + k;
    if (l16 == 0) {
      if (2 * p < m0) sigs[2 * p] = sqrt(nt);
      if (2 * p + 1 < m0) sigs[2 * p + 1] = sqrt(nb);
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < m0; j += JTHR) {
    const int q = desc_rank(sigs, m0, j);
    rk[j] = q;
    sorted[q] = sigs[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int t;
    const int cap = min(min(m0, d.r_int_max), d.T);
    if (d.forced && d.force[axis * d.nsub + s] > 0) {
      t = min(d.force[axis * d.nsub + s], cap);
    } else {
      const double tol = (d.rank_mode == 0) ? d.tol_aug_rel * sorted[0] : d.tol;
      t = max(r, tail_rank(sorted, m0, tol));
      if (t > cap) {
        t = cap;
        atomicAdd(d.clamps, 1ull);
        if (d.strict) atomicOr(d.flags, FLAG_RANK_CLAMP);
      }
    }
    if (t < 1) t = 1;
    sc.ival[0] = t;
    d.tdim[s] = t;
    if (t > d.tmax[s]) d.tmax[s] = t;
  }
  __syncthreads();
  const int t = sc.ival[0];
  const double s0 = sorted[0];
  for (int j = threadIdx.x; j < m0; j += JTHR) sm[d.oSig + j] = sorted[j];
  for (int j = threadIdx.x; j < t; j += JTHR)
    sm[d.oFill + j] = (s0 > 0.0 && sorted[j] > 1e-13 * s0) ? 0.0 : 1.0;
  // Coef[:, rank(c)] = b_c / sigma_c^2 for the kept columns
#pragma unroll
  for (int k = 0; k < PPG; ++k) {
    const int p = gi * PPG + k;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int col = 2 * p + half;
      if (col >= m0) continue;
      const int q = rk[col];
      if (q >= t) continue;
      const double sg = sigs[col];
      const bool ok = s0 > 0.0 && sg > 1e-13 * s0;
      const double isg2 = ok ? 1.0 / (sg * sg) : 0.0;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int row = l16 + 16 * i;
        if (row < m0) sm[d.oCoef + row + q * d.MA] = (half ? c.b[i][k] : c.t[i][k]) * isg2;
      }
    }
  }
}

__global__ __launch_bounds__(JTHR) void sw_aug_svd(Dev d, int axis, int sd0) {
  const int s = sd0 + blockIdx.x;
  const int m0 = m0_of(d, s, axis);
  extern __shared__ double lds[];
  __shared__ SmallScratch sc;
  if (m0 <= 64) aug_svd_body<2, 4>(d, s, axis, m0, lds, sc);
  else if (m0 <= 128) aug_svd_body<2, 8>(d, s, axis, m0, lds, sc);
  else aug_svd_body<3, 12>(d, s, axis, m0, lds, sc);
}

// Upwind split of the angular Galerkin matrix C (Appendix A: C = P diag(lambda)
// P^T, C+ = P diag(max(lambda, 0)) P^T, C- = P diag(min(lambda, 0)) P^T) for
// t <= 128 by the sign function (ns_abs), and the K-step coefficients
//   M0 = Am (I - nu C+ + nu C-), Mm = nu Am C+, Mp = -nu Am C-,
//   GLo = nu Am En C+, GHi = -nu Am Ep C-,
//   GLoN = nu S_lo Olo C+, GHiN = -nu S_hi Ohi C-,   Am = S Tm, nu = dt c / h.
__device__ void adv_prep_body(const Dev& d, int s, int axis, int t, double* lds, SmallScratch& sc) {
  const int lo = neighbour(d, s, axis, -1), hi = neighbour(d, s, axis, +1);
  const int r = d.rank[s], rl = lo >= 0 ? d.rank[lo] : 0, rh = hi >= 0 ? d.rank[hi] : 0;
  const int R = d.R, T = d.T;
  double* sm = small_of(d, s);
  double* Cl = lds;  // t x t, ld WLD
  const int pT = 0, pC = R * T, pEp = pC + T * T, pEn = pEp + T * T, pOlo = pEn + T * T, pOhi = pOlo + R * T;
  const int ngp = d.xgM;
  s_sum_partials(d, s, ngp, pT, R, r, t, sm + d.oTm, R, 1.0);
  s_sum_partials(d, s, ngp, pEp, t, t, t, sm + d.oEp, T, 1.0);
  s_sum_partials(d, s, ngp, pEn, t, t, t, sm + d.oEn, T, 1.0);
  s_sum_partials(d, s, ngp, pOlo, R, rl, t, sm + d.oOlo, R, 1.0);
  s_sum_partials(d, s, ngp, pOhi, R, rh, t, sm + d.oOhi, R, 1.0);
  s_sum_partials(d, s, ngp, pC, t, t, t, Cl, WLD, 1.0);
  __syncthreads();
  double* Cp = sm + d.oCp;
  double* Cn = sm + d.oCn;
  {
    // symmetric C in the workspace, then the sign-function split
    double* Cw = sm + d.oW4;
    double* Ab = sm + d.oW3;
    for (int idx = threadIdx.x; idx < t * t; idx += STHR) {
      const int i = idx % t, j = idx / t;
      Cw[i + j * T] = 0.5 * (Cl[i + j * WLD] + Cl[j + i * WLD]);
    }
    __syncthreads();
    ns_abs(Cw, sm + d.oW5, sm + d.oW1, sm + d.oW2, Ab, t, T, sc.red);
    for (int idx = threadIdx.x; idx < t * t; idx += STHR) {
      const int i = idx % t, j = idx / t;
      const double c = Cw[i + j * T], ab = 0.5 * (Ab[i + j * T] + Ab[j + i * T]);
      Cp[i + j * T] = 0.5 * (c + ab);
      Cn[i + j * T] = 0.5 * (c - ab);
    }
    __syncthreads();
  }
  const double nu = d.dt * d.c / d.h;
  const double* Sg = d.S + (int64_t)s * R * R;
  double* Am = sm + d.oAm;
  double* W1 = sm + d.oW1;
  double* W2 = sm + d.oW2;
  double* W3 = sm + d.oW3;
  gmm(Am, R, Sg, R, false, sm + d.oTm, R, false, r, t, r, 1.0, 0.0);
  gmm(W1, R, Am, R, false, Cp, T, false, r, t, t, 1.0, 0.0);
  gmm(W2, R, Am, R, false, Cn, T, false, r, t, t, 1.0, 0.0);
  for (int idx = threadIdx.x; idx < r * t; idx += STHR) {
    const int i = idx % r, j = idx / r;
    const int o = i + j * R;
    sm[d.oM0 + o] = Am[o] - nu * W1[o] + nu * W2[o];
    sm[d.oMm + o] = nu * W1[o];
    sm[d.oMp + o] = -nu * W2[o];
  }
  __syncthreads();
  gmm(W3, T, sm + d.oEn, T, false, Cp, T, false, t, t, t, 1.0, 0.0);
  gmm(sm + d.oGLo, R, Am, R, false, W3, T, false, r, t, t, nu, 0.0);
  gmm(W3, T, sm + d.oEp, T, false, Cn, T, false, t, t, t, 1.0, 0.0);
  gmm(sm + d.oGHi, R, Am, R, false, W3, T, false, r, t, t, -nu, 0.0);
  if (rl > 0) {
    gmm(W1, R, sm + d.oOlo, R, false, Cp, T, false, rl, t, t, 1.0, 0.0);
    gmm(sm + d.oGLoN, R, d.S + (int64_t)lo * R * R, R, false, W1, R, false, rl, t, rl, nu, 0.0);
  }
  if (rh > 0) {
    gmm(W2, R, sm + d.oOhi, R, false, Cn, T, false, rh, t, t, 1.0, 0.0);
    gmm(sm + d.oGHiN, R, d.S + (int64_t)hi * R * R, R, false, W2, R, false, rh, t, rh, -nu, 0.0);
  }
}

__global__ __launch_bounds__(STHR) void sw_adv_prep(Dev d, int axis, int sd0) {
  const int s = sd0 + blockIdx.x;
  const int t = d.tdim[s];
  extern __shared__ double lds[];
  __shared__ SmallScratch sc;
  adv_prep_body(d, s, axis, t, lds, sc);
}

// sw_rk_prep: the frozen ghost rows of the low and high faces,
//   Kb_lo = K0[low face] En + U_lo[its high face] S_lo Olo,
//   Kb_hi = K0[high face] Ep + U_hi[its low face] S_hi Ohi,
// with K0 = U Am (Am = S Tm), into d.ghost[s][side][j][f].
__global__ __launch_bounds__(STHR) void sw_rk_prep(Dev d, int axis, int sd0) {
  const int s = sd0 + blockIdx.x;
  const int lo = neighbour(d, s, axis, -1), hi = neighbour(d, s, axis, +1);
  const int r = d.rank[s], rl = lo >= 0 ? d.rank[lo] : 0, rh = hi >= 0 ? d.rank[hi] : 0;
  const int t = d.tdim[s];
  const int R = d.R, T = d.T, N = d.N;
  double* sm = small_of(d, s);
  double* AEn = sm + d.oW1;  // r x t, ld T
  double* AEp = sm + d.oW2;
  double* SOl = sm + d.oW3;  // rl x t
  double* SOh = sm + d.oW4;  // rh x t
  gmm(AEn, T, sm + d.oAm, R, false, sm + d.oEn, T, false, r, t, t, 1.0, 0.0);
  gmm(AEp, T, sm + d.oAm, R, false, sm + d.oEp, T, false, r, t, t, 1.0, 0.0);
  if (rl > 0) gmm(SOl, T, d.S + (int64_t)lo * R * R, R, false, sm + d.oOlo, R, false, rl, t, rl, 1.0, 0.0);
  if (rh > 0) gmm(SOh, T, d.S + (int64_t)hi * R * R, R, false, sm + d.oOhi, R, false, rh, t, rh, 1.0, 0.0);
  const int F = face_len(d, axis);
  const double* U = d.U + (int64_t)s * N * R;
  const double* Ul = lo >= 0 ? d.U + (int64_t)lo * N * R : U;
  const double* Uh = hi >= 0 ? d.U + (int64_t)hi * N * R : U;
  double* glo = d.ghost + (int64_t)(2 * s) * T * d.face;
  double* ghi = glo + (int64_t)T * d.face;
  for (int idx = threadIdx.x; idx < F * t; idx += STHR) {
    const int f = idx % F, j = idx / F;
    const int pl = face_cell(d, axis, false, f), ph = face_cell(d, axis, true, f);
    double a = 0.0, b = 0.0;
    for (int k = 0; k < r; ++k) {
      a = fma(U[(int64_t)k * N + pl], AEn[k + j * T], a);
      b = fma(U[(int64_t)k * N + ph], AEp[k + j * T], b);
    }
    for (int k = 0; k < rl; ++k) a = fma(Ul[(int64_t)k * N + ph], SOl[k + j * T], a);
    for (int k = 0; k < rh; ++k) b = fma(Uh[(int64_t)k * N + pl], SOh[k + j * T], b);
    glo[(int64_t)j * d.face + f] = a;
    ghi[(int64_t)j * d.face + f] = b;
  }
}

// S-step (eq. advx_evolS, integrated with the opposite sign) and the L-step
// coefficients, as in the narrow plan (Q = h U^1, frozen boundary data):
//   BKlo = Xlo (Am En) + Xln (S_lo Olo),  BKhi = Xhi (Am Ep) + Xhn (S_hi Ohi),
//   H-(S) = Gm S - BKlo,  H+(S) = Gp S + BKhi,  Gm = -Gp^T,
//   S1 = h Racc,  S2 = S1 + dt c (H-(S1) C+ + H+(S1) C-),
//   P0 = S2^T, Pm = -dt c H-(S2)^T, Pp = -dt c H+(S2)^T.
__global__ __launch_bounds__(STHR) void sw_adv_sstep(Dev d, int axis, int sd0) {
  const int s = sd0 + blockIdx.x;
  const int lo = neighbour(d, s, axis, -1), hi = neighbour(d, s, axis, +1);
  const int r = d.rank[s], rl = lo >= 0 ? d.rank[lo] : 0, rh = hi >= 0 ? d.rank[hi] : 0;
  const int t = d.tdim[s];
  const int R = d.R, T = d.T;
  double* sm = small_of(d, s);
  const double ih = 1.0 / d.h;
  double* Gm = sm + d.oGm;
  double* Gp = sm + d.oGp;
  double* Xlo = sm + d.oW1;
  double* Xhi = sm + d.oW2;
  double* Xln = sm + d.oW3;
  double* Xhn = sm + d.oW4;
  const int oX = 2 * T * T, ngp = d.xgN;
  s_sum_partials(d, s, ngp, 0, t, t, t, Gp, T, ih);
  s_sum_partials(d, s, ngp, oX, T, t, r, Xlo, T, 1.0);
  s_sum_partials(d, s, ngp, oX + T * R, T, t, r, Xhi, T, 1.0);
  s_sum_partials(d, s, ngp, oX + 2 * T * R, T, t, rl, Xln, T, 1.0);
  s_sum_partials(d, s, ngp, oX + 3 * T * R, T, t, rh, Xhn, T, 1.0);
  __syncthreads();
  double* W5 = sm + d.oW5;
  double* W6 = sm + d.oW6;
  double* BKlo = sm + d.oBKlo;
  double* BKhi = sm + d.oBKhi;
  double* S1 = sm + d.oS1;
  double* S2 = sm + d.oS2;
  const double* Slo = lo >= 0 ? d.S + (int64_t)lo * R * R : d.S;
  const double* Shi = hi >= 0 ? d.S + (int64_t)hi * R * R : d.S;
  gmm(W5, R, sm + d.oAm, R, false, sm + d.oEn, T, false, r, t, t, 1.0, 0.0);
  gmm(S1, T, sm + d.oAm, R, false, sm + d.oEp, T, false, r, t, t, 1.0, 0.0);
  gmm(BKlo, T, Xlo, T, false, W5, R, false, t, t, r, 1.0, 0.0);
  gmm(BKhi, T, Xhi, T, false, S1, T, false, t, t, r, 1.0, 0.0);
  if (rl > 0) {
    gmm(W6, R, Slo, R, false, sm + d.oOlo, R, false, rl, t, rl, 1.0, 0.0);
    gmm(BKlo, T, Xln, T, false, W6, R, false, t, t, rl, 1.0, 1.0);
  }
  if (rh > 0) {
    gmm(S2, T, Shi, R, false, sm + d.oOhi, R, false, rh, t, rh, 1.0, 0.0);
    gmm(BKhi, T, Xhn, T, false, S2, T, false, t, t, rh, 1.0, 1.0);
  }
  for (int idx = threadIdx.x; idx < t * t; idx += STHR) {
    const int i = idx % t, j = idx / t;
    S1[i + j * T] = d.h * sm[d.oRacc + i + j * T];
    Gm[i + j * T] = -Gp[j + i * T];
  }
  __syncthreads();
  double* Hm = W5;
  double* Hp = W6;
  // S-step: S' = c ((Gm S - BKlo) C+ + (Gp S + BKhi) C-), one Euler step, or
  // RK4 in the nested form S2 = S1 + dt f(S1 + dt/2 f(S1 + dt/3 f(S1 + dt/4 f(S1))))
  // (stage outputs alternate between S2 and W1, the last one is copied to S2)
  const int nst = d.rk4 ? 4 : 1;
  const double* Sin = S1;
  for (int stg = 0; stg < nst; ++stg) {
    const double al = d.dt / (double)(nst - stg);
    double* Sout = (stg & 1) ? Xlo : S2;
    gmm(Hm, T, Gm, T, false, Sin, T, false, t, t, t, 1.0, 0.0);
    gmm(Hp, T, Gp, T, false, Sin, T, false, t, t, t, 1.0, 0.0);
    for (int idx = threadIdx.x; idx < t * t; idx += STHR) {
      const int o = (idx % t) + (idx / t) * T;
      Hm[o] -= BKlo[o];
      Hp[o] += BKhi[o];
      Sout[o] = S1[o];
    }
    __syncthreads();
    const double dc = al * d.c;
    gmm(Sout, T, Hm, T, false, sm + d.oCp, T, false, t, t, t, dc, 1.0);
    gmm(Sout, T, Hp, T, false, sm + d.oCn, T, false, t, t, t, dc, 1.0);
    Sin = Sout;
  }
  if (Sin != S2) {
    for (int idx = threadIdx.x; idx < t * t; idx += STHR) {
      const int o = (idx % t) + (idx / t) * T;
      S2[o] = Sin[o];
    }
    __syncthreads();
  }
  const double dc = d.dt * d.c;
  gmm(Hm, T, Gm, T, false, S2, T, false, t, t, t, 1.0, 0.0);
  gmm(Hp, T, Gp, T, false, S2, T, false, t, t, t, 1.0, 0.0);
  for (int idx = threadIdx.x; idx < t * t; idx += STHR) {
    const int i = idx % t, j = idx / t;
    const int o = i + j * T, ot = j + i * T;
    sm[d.oP0 + ot] = S2[o];
    sm[d.oPm + ot] = -dc * (Hm[o] - BKlo[o]);
    sm[d.oPp + ot] = -dc * (Hp[o] + BKhi[o]);
  }
  if (d.rk4) {
    // L-step of direction q in the class of the sign of w = Omega_q: with
    // L = V-hat_q X, X' = w (X A + B) (A+ = -c Gm^T, A- = -c Gp^T), whose RK4
    // step is the degree-4 Taylor polynomial X1 = sum_j w^j N_j with
    // N0 = S2^T, N1 = dt (S2^T A + B) (the Euler Pm / Pp above) and
    // N_{j+1} = dt / (j + 1) N_j A: N2..N4 of the + class into W1, W3, W5,
    // of the - class into W2, W4, W6
    __syncthreads();
    double* Np[4] = {sm + d.oPm, sm + d.oW1, sm + d.oW3, sm + d.oW5};
    double* Nn[4] = {sm + d.oPp, sm + d.oW2, sm + d.oW4, sm + d.oW6};
    for (int j = 1; j < 4; ++j) {
      const double a = -d.c * d.dt / (double)(j + 1);
      gmm(Np[j], T, Np[j - 1], T, false, Gm, T, true, t, t, t, a, 0.0);
      gmm(Nn[j], T, Nn[j - 1], T, false, Gp, T, true, t, t, t, a, 0.0);
    }
  }
}

// Truncation (Algorithm 5) for t <= 128: S3 = RL^T, ring Jacobi with the
// rotations accumulated (S3 J = U~ Sigma, V~ = J), the rank rule, and the
// rotations Bu = U~[:, :r'] / h, Bv = V~[:, :r'] of the final products;
// S = diag(sigma[:r']) goes into the state and r' into rnew.
template <int PPG, int RPL>
__device__ __forceinline__ void trunc_body(const Dev& d, int s, int axis, int t, double* lds, SmallScratch& sc) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane >> 2, gi = 4 * wave + (lane & 3);
  const int R = d.R, T = d.T;
  double* sm = small_of(d, s);
  double* sigs = sc.v0;
  double* sorted = sc.v1;
  int* rk = sc.i0;
  const double* RL = sm + d.oRacc;
  GRing<PPG, RPL, true, RPL> c;
#pragma unroll
  for (int i = 0; i < RPL; ++i)
#pragma unroll
    for (int k = 0; k < PPG; ++k) {
      const int row = l16 + 16 * i, p = gi * PPG + k;
      const int ct = 2 * p, cb = 2 * p + 1;
      c.t[i][k] = (row < t && ct < t) ? RL[ct + row * T] : 0.0;   // S3[row][col] = RL[col][row]
      c.b[i][k] = (row < t && cb < t) ? RL[cb + row * T] : 0.0;
      c.jt[i][k] = (row == ct && ct < t) ? 1.0 : 0.0;
      c.jb[i][k] = (row == cb && cb < t) ? 1.0 : 0.0;
    }
#pragma unroll
  for (int k = 0; k < PPG; ++k) c.nt[k] = c.nb[k] = 0.0;
  gring_jacobi<PPG, RPL, true, RPL>(d, c, t, 1e-14, 1e-15, 40, lds, sc.red, sc.rotflag);
#pragma unroll
  for (int k = 0; k < PPG; ++k) {
    double nt = 0.0, nb = 0.0;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      nt = fma(c.t[i][k], c.t[i][k], nt);
      nb = fma(c.b[i][k], c.b[i][k], nb);
    }
    nt = class_sum16(nt);
    nb = class_sum16(nb);
    const int p = gi * PPG + k;
    if (l16 == 0) {
      if (2 * p < t) sigs[2 * p] = sqrt(nt);
      if (2 * p + 1 < t) sigs[2 * p + 1] = sqrt(nb);
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < t; j += JTHR) {
    const int q = desc_rank(sigs, t, j);
    rk[j] = q;
    sorted[q] = sigs[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int rp;
    const int cap = min(min(d.r_max, t), R);
    if (d.forced && d.force[2 * d.nsub + axis * d.nsub + s] > 0) {
      rp = min(d.force[2 * d.nsub + axis * d.nsub + s], min(t, R));
    } else if (d.rank_mode == 0) {
      rp = min(d.r_fixed, min(t, R));
    } else {
      rp = max(d.r_min, tail_rank(sorted, t, d.tol));
      if (rp > cap) {
        rp = cap;
        atomicAdd(d.clamps, 1ull);
        if (d.strict) atomicOr(d.flags, FLAG_RANK_CLAMP);
      }
    }
    if (rp < 1) rp = 1;
    sc.ival[0] = rp;
    d.rnew[s] = rp;
    sc.ival[1] = 0;
  }
  __syncthreads();
  const int rp = sc.ival[0];
  const double s0 = sorted[0];
  const double ih = 1.0 / d.h;
  double* Ut = sm + d.oBu;
  double* Bv = sm + d.oBv;
#pragma unroll
  for (int k = 0; k < PPG; ++k) {
    const int p = gi * PPG + k;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int col = 2 * p + half;
      if (col >= t) continue;
      const int q = rk[col];
      if (q >= rp) continue;
      const double sg = sigs[col];
      const bool ok = s0 > 0.0 && sg > 1e-13 * s0;
      if (!ok && l16 == 0) sc.ival[1] = 1;
      const double isg = ok ? 1.0 / sg : 0.0;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int row = l16 + 16 * i;
        if (row < t) {
          const double b = half ? c.b[i][k] : c.t[i][k];
          const double v = half ? c.jb[i][k] : c.jt[i][k];
          Ut[row + q * T] =
              ok ? b * isg : hash_unit(((uint64_t)s << 40) ^ ((uint64_t)(q + 1000) << 24) ^ (uint64_t)row);
          Bv[row + q * T] = v;
        }
      }
    }
  }
  __syncthreads();
  // completed columns are made orthonormal to the others (two passes of
  // modified Gram-Schmidt)
  if (sc.ival[1]) {
    for (int pass = 0; pass < 2; ++pass)
      for (int j = 0; j < rp; ++j) {
        for (int k = 0; k < j; ++k) {
          double part = 0.0;
          for (int i = threadIdx.x; i < t; i += JTHR) part = fma(Ut[i + k * T], Ut[i + j * T], part);
          const double dot = s_sum(part, sc.red);
          for (int i = threadIdx.x; i < t; i += JTHR) Ut[i + j * T] -= dot * Ut[i + k * T];
          __syncthreads();
        }
        double part = 0.0;
        for (int i = threadIdx.x; i < t; i += JTHR) part = fma(Ut[i + j * T], Ut[i + j * T], part);
        const double nrm = sqrt(s_sum(part, sc.red));
        const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
        for (int i = threadIdx.x; i < t; i += JTHR) Ut[i + j * T] *= inv;
        __syncthreads();
      }
  }
  for (int idx = threadIdx.x; idx < t * rp; idx += JTHR) {
    const int i = idx % t, j = idx / t;
    Ut[i + j * T] *= ih;
  }
  double* Sg = d.S + (int64_t)s * R * R;
  for (int idx = threadIdx.x; idx < R * R; idx += JTHR) {
    const int i = idx % R, j = idx / R;
    Sg[idx] = (i == j && i < rp) ? sorted[i] : 0.0;
  }
  if (threadIdx.x < rp && !isfinite(sorted[threadIdx.x])) atomicOr(d.flags, FLAG_NONFINITE);
}

__global__ __launch_bounds__(JTHR) void sw_trunc(Dev d, int axis, int sd0) {
  const int s = sd0 + blockIdx.x;
  const int t = d.tdim[s];
  extern __shared__ double lds[];
  __shared__ SmallScratch sc;
  if (t <= 64) trunc_body<2, 4>(d, s, axis, t, lds, sc);
  else trunc_body<2, 8>(d, s, axis, t, lds, sc);
}

// m = V^T w (eq. coll_evolK) for stored ranks up to 64: one wavefront per
// column, lanes striding over the directions, summed in a fixed order.
__global__ __launch_bounds__(STHR) void sw_coll_prep(Dev d, int sd0) {
  const int s = sd0 + blockIdx.x;
  const int r = d.rank[s];
  const int M = d.M, R = d.R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double* Vs = d.V + (int64_t)s * M * R;
  for (int a = wave; a < r; a += SNW) {
    double acc = 0.0;
    for (int q = lane; q < M; q += 64) acc = fma(Vs[(int64_t)a * M + q], d.w[q], acc);
    acc = wave_sum(acc);
    if (lane == 0) small_of(d, s)[d.oMv + a] = acc;
  }
}

// ============================================================================
// launchers
// ============================================================================
namespace {
template <int V>
using wic = std::integral_constant<int, V>;
template <class T>
struct wtag {
  using type = T;
};

template <class Fn>
void w_with_prec(int prec, bool exact, Fn f) {
  if (prec == DD_PREC_FP64) f(wtag<double>{}, wic<0>{});
  else if (exact) f(wtag<float>{}, wic<0>{});
  else if (prec == DD_PREC_MIXED_FP32) f(wtag<float>{}, wic<1>{});
  else f(wtag<float>{}, wic<2>{});
}

// the dynamic LDS of a kernel may exceed the default limit only after this
// attribute is set; it is set once per kernel (at handle creation), outside
// any graph capture
void w_allow(const void* fn) {
  (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
}

int w_dim_cap(const Dev& d, int which) { return which == DIM_M0 ? d.MA : (which == DIM_T ? d.T : d.R); }

constexpr size_t AUG_RING_LDS = sizeof(double) * gring_lds_doubles<GRing<3, 12, false, 1>::CW>();
constexpr size_t TRUNC_RING_LDS = sizeof(double) * gring_lds_doubles<GRing<2, 8, true, 8>::CW>();

// every small kernel's dynamic LDS plus its static scratch fits the 160 KB
// of a compute unit
constexpr size_t LDS_CU = 160 * 1024;
constexpr size_t AUG_LDS = sizeof(double) * (size_t)WCAP_A * (WCAP_A + 1) / 2;
static_assert(AUG_RING_LDS <= AUG_LDS, "ring buffer of the augmentation SVD");
static_assert(AUG_LDS + sizeof(SmallScratch) <= LDS_CU, "LDS of sw_aug_svd");
static_assert(TRUNC_RING_LDS + sizeof(SmallScratch) <= LDS_CU, "LDS of sw_trunc");
static_assert(sizeof(double) * (size_t)WLD * WCAP_T + sizeof(SmallScratch) <= LDS_CU, "LDS of sw_chol/adv_prep");
}  // namespace

void launch_w_gemm(const Dev& d, int axis, int sd0, int nsd, const void* X, bool x64, int64_t xsd, int rows,
                   int kdim, int ndim, int boff, int bld, void* Y, bool y64, int64_t ysd, const double* rowscale,
                   int fill_off, bool rows_are_cells, bool exact, hipStream_t st, bool set_rank, int skip_off) {
  const int nwg = rows_are_cells ? d.nwgN : d.nwgM;
  constexpr int NCB = 4;
  const int nz = wdiv(w_dim_cap(d, ndim), 16 * NCB);
  const int ng = wdiv(w_dim_cap(d, kdim), 64);
  auto go = [&](auto ti, auto to, auto pc) {
    using SI = typename decltype(ti)::type;
    using SO = typename decltype(to)::type;
    constexpr int P = decltype(pc)::value;
    const size_t lds = sizeof(typename Prec<P>::F) * (size_t)ng * 16 * NCB * 64;
    hipLaunchKernelGGL((kw_gemm<SI, SO, P, NCB>), dim3(nwg, nsd, nz), dim3(WTHR), lds, st, d, axis, sd0, X, xsd,
                       rows, kdim, ndim, boff, bld, Y, ysd, rowscale, fill_off, set_rank ? 1 : 0, skip_off);
  };
  w_with_prec(d.prec, exact, [&](auto ts, auto pc) {
    using W = typename decltype(ts)::type;
    if (x64 && y64) go(wtag<double>{}, wtag<double>{}, pc);
    else if (x64) go(wtag<double>{}, wtag<W>{}, pc);
    else if (y64) go(wtag<W>{}, wtag<double>{}, pc);
    else go(wtag<W>{}, wtag<W>{}, pc);
  });
}

void launch_w_aug_form(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  const size_t lds = sizeof(double) * 16 * 4 * 64;
  hipLaunchKernelGGL(kw_aug_form, dim3(d.nwgM, nsd, 3), dim3(WTHR), lds, st, d, axis, sd0);
}

void launch_w_kstep(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  const int nz = wdiv(d.T, 32);
  w_with_prec(d.prec, false, [&](auto ts, auto pc) {
    using S = typename decltype(ts)::type;
    constexpr int P = decltype(pc)::value;
    const size_t lds = sizeof(typename Prec<P>::F) * 7 * 16 * 2 * 64;
    hipLaunchKernelGGL((kw_kstep<S, P>), dim3(d.nwgN, nsd, nz), dim3(WTHR), lds, st, d, axis, sd0);
  });
}

void launch_w_rk_prep(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  hipLaunchKernelGGL(sw_rk_prep, dim3(nsd), dim3(STHR), 0, st, d, axis, sd0);
}

void launch_w_rk_kstep(const Dev& d, int axis, int sd0, int nsd, double alpha, const void* in, void* out,
                       hipStream_t st) {
  hipLaunchKernelGGL(kw_rk_kstep, dim3(wdiv(d.N, 64), nsd, wdiv(d.T, RKC)), dim3(WTHR), 0, st, d, axis, sd0, alpha,
                     (const double*)in, (double*)out);
}

void launch_w_lstep(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  const int nz = wdiv(d.T, 32);
  w_with_prec(d.prec, false, [&](auto ts, auto pc) {
    using S = typename decltype(ts)::type;
    constexpr int P = decltype(pc)::value;
    if (d.rk4) {
      // RK4 (FP64 only): nine coefficient matrices, 16 output columns per workgroup
      const size_t lds = sizeof(double) * 9 * (WCAP_T / 64) * 16 * 1 * 64;
      hipLaunchKernelGGL((kw_lstep<double, 0, 9, 1>), dim3(d.nwgM, nsd, wdiv(d.T, 16)), dim3(WTHR), lds, st, d,
                         axis, sd0);
      return;
    }
    const size_t lds = sizeof(typename Prec<P>::F) * 3 * (WCAP_T / 64) * 16 * 2 * 64;
    hipLaunchKernelGGL((kw_lstep<S, P, 3, 2>), dim3(d.nwgM, nsd, nz), dim3(WTHR), lds, st, d, axis, sd0);
  });
}

void launch_w_coll_kstep(const Dev& d, int sd0, int nsd, hipStream_t st) {
  const int nz = wdiv(d.R, 32);
  w_with_prec(d.prec, false, [&](auto ts, auto pc) {
    using S = typename decltype(ts)::type;
    constexpr int P = decltype(pc)::value;
    hipLaunchKernelGGL((kw_coll_kstep<S, P>), dim3(d.nwgN, nsd, nz), dim3(WTHR), 0, st, d, sd0);
  });
}

void launch_w_xgram(const Dev& d, int axis, int sd0, int nsd, XJobs jobs, bool cells, int np, hipStream_t st) {
  int z = 0;
  for (int q = 0; q < jobs.n; ++q) {
    XJob& J = jobs.j[q];
    J.zbase = z;
    z += J.sym ? J.pa * (J.pa + 1) / 2 : J.pa * J.pb;
    J.rows_cells = cells ? 1 : 0;
  }
  if (d.prec == DD_PREC_FP64)
    hipLaunchKernelGGL(kw_xgram<double>, dim3(np, nsd, z), dim3(XTHR), 0, st, d, axis, sd0,
                       jobs);
  else
    hipLaunchKernelGGL(kw_xgram<float>, dim3(np, nsd, z), dim3(XTHR), 0, st, d, axis, sd0,
                       jobs);
}

void launch_w_chol(const Dev& d, int axis, int sd0, int nsd, int ndim, int rows, int ngp, int acc_mode,
                   double bscale, int oRinv, int oRacc, int ld, bool near, hipStream_t st, int skip_mode) {
  const size_t lds = sizeof(double) * (size_t)WLD * WCAP_T;
  hipLaunchKernelGGL(sw_chol, dim3(nsd), dim3(STHR), lds, st, d, axis, sd0, ndim, rows, ngp, acc_mode, bscale,
                     oRinv, oRacc, ld, near ? 1 : 0, skip_mode);
}

void launch_w_aug_svd(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  const size_t lds = std::max(AUG_LDS, AUG_RING_LDS);
  hipLaunchKernelGGL(sw_aug_svd, dim3(nsd), dim3(JTHR), lds, st, d, axis, sd0);
}

void launch_w_adv_prep(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  const size_t lds = sizeof(double) * (size_t)WLD * WCAP_T;
  hipLaunchKernelGGL(sw_adv_prep, dim3(nsd), dim3(STHR), lds, st, d, axis, sd0);
}

void launch_w_adv_sstep(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  hipLaunchKernelGGL(sw_adv_sstep, dim3(nsd), dim3(STHR), 0, st, d, axis, sd0);
}

void launch_w_trunc(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  const size_t lds = TRUNC_RING_LDS;
  hipLaunchKernelGGL(sw_trunc, dim3(nsd), dim3(JTHR), lds, st, d, axis, sd0);
}

void launch_w_coll_prep(const Dev& d, int sd0, int nsd, hipStream_t st) {
  hipLaunchKernelGGL(sw_coll_prep, dim3(nsd), dim3(STHR), 0, st, d, sd0);
}

void init_wide_kernels() {
  for (int prec = 0; prec < 3; ++prec)
    for (int exact = 0; exact < 2; ++exact)
      w_with_prec(prec, exact != 0, [&](auto ts, auto pc) {
        using W = typename decltype(ts)::type;
        constexpr int P = decltype(pc)::value;
        w_allow((const void*)kw_gemm<double, double, P, 4>);
        w_allow((const void*)kw_gemm<double, W, P, 4>);
        w_allow((const void*)kw_gemm<W, double, P, 4>);
        w_allow((const void*)kw_gemm<W, W, P, 4>);
        w_allow((const void*)kw_kstep<W, P>);
        w_allow((const void*)kw_lstep<W, P, 3, 2>);
      });
  w_allow((const void*)kw_aug_form);
  w_allow((const void*)sw_chol);
  w_allow((const void*)sw_aug_svd);
  w_allow((const void*)sw_adv_prep);
  w_allow((const void*)sw_trunc);
  w_allow((const void*)kw_lstep<double, 0, 9, 1>);
  (void)hipGetLastError();
}

}  // namespace dd
