// Tall-skinny kernels of the DD-DLRA step on the FP64 matrix cores.
//
// Every launch covers all subdomains of a batch (blockIdx.y).  Inside a
// subdomain the rows (cells or directions) are cut into strips of 16; strip
// st belongs to wavefront st mod (4 gridDim.x) of the workgroups blockIdx.x,
// so a workgroup takes 64 consecutive rows at a time and no barrier is
// needed inside the strip loop.  The loop is software-pipelined: the global
// loads of a wavefront's next strip are issued before the matrix-core
// instructions of the current one, so load latency overlaps the products
// (the grids are sized so that one to a few workgroups per compute unit
// cover the whole batch, and each wavefront walks many strips).  Reductions over rows (Gram and
// Galerkin matrices) stay in the wavefronts' accumulators, are summed over
// the workgroup in a fixed order and leave one partial per workgroup; the
// small per-subdomain kernels add the partials in a fixed order, so results
// are bitwise reproducible.
//
// Memory layout (per subdomain, column-major, one column contiguous):
//   cells  p = iy*lnx + ix  -> x-neighbours at p+-1, y-neighbours at p+-lnx
//   directions q            -> rows of V, V-hat, L
#include <algorithm>
#include <type_traits>

#include "dd_dlra.h"
#include "dd_mfma.h"

namespace dd {

constexpr int CAPR = 21;  // largest stored rank (3 * CAPR <= CAP)

__host__ __device__ constexpr int ceil_div(int a, int b) { return (a + b - 1) / b; }

// ----------------------------------------------------------------------------
// Augmentation matrix (Algorithm 4, step 1), weighted by sqrt(w) so that the
// plain Gram matrix is L0^T W L0:
//   A[q, :] = sqrt(w_q) [ V[q,:] S^T | V_lo[q,:] S_lo^T | V_hi[q,:] S_hi^T ]
// formed as one product [V | V_lo | V_hi] blockdiag(S^T, S_lo^T, S_hi^T);
// leaves the partial Gram matrix A^T A.
// ----------------------------------------------------------------------------
template <class S, int P, int NCB, int KS>
__global__ __launch_bounds__(NTHR) void k_aug_form(Dev d, int axis, int sd0) {
  using F = typename Prec<P>::F;
  using Acc = typename Prec<P>::Acc;
  constexpr int LD = strip_ld<NCB>();
  constexpr int NB = NCB * (NCB + 1) / 2;
  const int s = sd0 + blockIdx.y;
  const int nb[3] = {s, neighbour(d, s, axis, -1), neighbour(d, s, axis, +1)};
  int rb[3];
  for (int b = 0; b < 3; ++b) rb[b] = nb[b] >= 0 ? d.rank[nb[b]] : 0;
  const int c1 = rb[0], c2 = rb[0] + rb[1];
  const int m0 = rb[0] + rb[1] + rb[2];
  const int M = d.M, R = d.R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;

  extern __shared__ double lds[];
  F* Bf = reinterpret_cast<F*>(lds);                                  // KS * NCB fragments
  double* Ys = lds + frag_doubles<P>(KS * NCB * 64) + wave * 16 * LD;  // wavefront strip
  for (int idx = threadIdx.x; idx < KS * NCB * 64; idx += NTHR) {
    const int l = idx & 63, f = idx >> 6, cb = f % NCB, u = f / NCB;
    const int kc = sub_col<P>(u, l >> 4), col = 16 * cb + (l & 15);
    double v = 0.0;
    if (kc < m0 && col < m0) {
      const int bk = kc < c1 ? 0 : (kc < c2 ? 1 : 2);
      const int bc = col < c1 ? 0 : (col < c2 ? 1 : 2);
      if (bk == bc) {
        const int off = bk == 0 ? 0 : (bk == 1 ? c1 : c2);
        v = d.S[(int64_t)nb[bk] * R * R + (col - off) + (int64_t)(kc - off) * R];
      }
    }
    Bf[idx] = (F)v;
  }
  __syncthreads();

  const double* Vb[3];
  for (int b = 0; b < 3; ++b) Vb[b] = nb[b] >= 0 ? d.V + (int64_t)nb[b] * M * R : d.V;
  S* As = (S*)d.A + (int64_t)s * M * d.MA;
  dbl4 g[NB];
  zero_acc<NB>(g);
  const int nst = ceil_div(M, 16);
  const int stride = gridDim.x * NW;
  F xn[KS];
  // loads never branch: indices are clamped to valid ones and the value of
  // an absent entry is replaced by zero
  auto load = [&](int st_) {
    const int q_ = st_ * 16 + l16;
    const int qc = q_ < M ? q_ : M - 1;
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      const int kc = sub_col<P>(u, kq);
      const bool in = q_ < M && kc < m0;
      const int kk = in ? kc : 0;
      const int bk = kk < c1 ? 0 : (kk < c2 ? 1 : 2);
      const int off = bk == 0 ? 0 : (bk == 1 ? c1 : c2);
      const double v = Vb[bk][(int64_t)(kk - off) * M + qc];
      xn[u] = in ? (F)v : (F)0;
    }
  };
  int st = blockIdx.x * NW + wave;
  if (st < nst) load(st);
  for (; st < nst; st += stride) {
    const int q = st * 16 + l16;
    const bool rin = q < M;
    F xv[KS];
#pragma unroll
    for (int u = 0; u < KS; ++u) xv[u] = xn[u];
    if (st + stride < nst) load(st + stride);
    Acc acc[NCB];
    zero_prod<P>(acc, NCB);
    prod_acc<P, NCB, KS>(acc, Bf, xv);
    const double swq = rin ? d.sw[q] : 0.0;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = out_col<P>(cb, v, kq);
        const S val = (S)((double)acc[cb][v] * swq);
        if (rin && j < m0) As[(int64_t)j * M + q] = val;
        Ys[l16 * LD + j] = (double)val;
      }
    }
    wave_sync();
    strip_gram<NCB, LD>(g, Ys);
    wave_sync();
  }
  wg_reduce_acc<NB>(g, lds);
  if (wave == 0) store_gram<NCB>(g, gpart_of(d, s) + (int64_t)blockIdx.x * d.gpTile, m0, 1.0);
}

// ----------------------------------------------------------------------------
// Generic tall-skinny product Y = diag(rowscale) X B with an optional
// partial Gram matrix of Y.  X is rows x k, B is k x n (small workspace,
// leading dimension bld).  Columns flagged in the fill mask are replaced by
// deterministic pseudo-random values (used to complete a basis where the
// data carry no information).  With set_rank, the first workgroup of each
// subdomain also commits the truncated rank (the product reads only the
// augmented and new ranks, never the current one).  With skip_off >= 0, a
// subdomain whose skip slot is set (B is the identity, Y is X) does nothing.
// ----------------------------------------------------------------------------
template <class SI, class S, int P, int NCB, int KS>
__global__ __launch_bounds__(NTHR) void k_gemm(Dev d, int axis, int sd0, const void* X, int64_t xsd, int rows,
                                               int kdim, int ndim, int boff, int bld, void* Y, int64_t ysd,
                                               const double* rowscale, int gram, int fill_off, int set_rank,
                                               int skip_off) {
  using F = typename Prec<P>::F;
  using Acc = typename Prec<P>::Acc;
  constexpr int LD = strip_ld<NCB>();
  const int s = sd0 + blockIdx.y;
  const int k = dim_of(d, s, axis, kdim);
  const int n = dim_of(d, s, axis, ndim);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  extern __shared__ double lds[];
  F* Bf = reinterpret_cast<F*>(lds);
  double* Ys = lds + frag_doubles<P>(KS * NCB * 64) + wave * 16 * LD;
  __shared__ int fillm[16 * NCB];
  const double* sm = small_of(d, s);
  if (skip_off >= 0 && sm[skip_off] != 0.0) return;  // identity in place
  for (int idx = threadIdx.x; idx < KS * NCB * 64; idx += NTHR) {
    const int l = idx & 63, f = idx >> 6, cb = f % NCB, u = f / NCB;
    const int kc = sub_col<P>(u, l >> 4), col = 16 * cb + (l & 15);
    Bf[idx] = (kc < k && col < n) ? (F)sm[boff + kc + col * bld] : (F)0;
  }
  for (int j = threadIdx.x; j < 16 * NCB; j += NTHR)
    fillm[j] = (fill_off >= 0 && j < n) ? (sm[fill_off + j] != 0.0) : 0;
  if (set_rank && blockIdx.x == 0 && threadIdx.x == 0) d.rank[s] = d.rnew[s];
  __syncthreads();

  const SI* Xsd = (const SI*)X + (int64_t)s * xsd;
  S* Ysd = (S*)Y + (int64_t)s * ysd;
  const int nst = ceil_div(rows, 16);
  const int stride = gridDim.x * NW;
  // NC output column blocks and KSR sub-steps are issued: a subdomain whose
  // operands have at most one instruction's live columns and 16 output
  // columns takes the short instance
  auto run = [&](auto nc_c, auto ks_c) {
    constexpr int NC = decltype(nc_c)::value, KSR = decltype(ks_c)::value;
    constexpr int NBR = NC * (NC + 1) / 2;
    dbl4 g[NBR];
    zero_acc<NBR>(g);
    F xn[KSR];
    auto load = [&](int st_) {
      const int row_ = st_ * 16 + l16;
      const int rc = row_ < rows ? row_ : rows - 1;
#pragma unroll
      for (int u = 0; u < KSR; ++u) {
        const int kc = sub_col<P>(u, kq);
        const bool in = row_ < rows && kc < k;
        const SI v = Xsd[(int64_t)(in ? kc : 0) * rows + rc];
        xn[u] = in ? (F)v : (F)0;
      }
    };
    int st = blockIdx.x * NW + wave;
    if (st < nst) load(st);
    for (; st < nst; st += stride) {
      const int row = st * 16 + l16;
      const bool rin = row < rows;
      F xv[KSR];
#pragma unroll
      for (int u = 0; u < KSR; ++u) xv[u] = xn[u];
      if (st + stride < nst) load(st + stride);
      Acc acc[NC];
      zero_prod<P>(acc, NC);
      prod_acc<P, NC, KSR, NCB>(acc, Bf, xv);
      const double rs = (rowscale != nullptr && rin) ? rowscale[row] : 1.0;
#pragma unroll
      for (int cb = 0; cb < NC; ++cb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = out_col<P>(cb, v, kq);
          double val = (double)acc[cb][v] * rs;
          if (fillm[j]) val = hash_unit(((uint64_t)s << 40) ^ ((uint64_t)j << 24) ^ (uint64_t)row);
          if (!rin) val = 0.0;
          const S sv = (S)val;
          if (rin && j < n) Ysd[(int64_t)j * rows + row] = sv;
          if (gram) Ys[l16 * LD + j] = (double)sv;
        }
      }
      if (gram) {
        wave_sync();
        strip_gram<NC, LD>(g, Ys);
        wave_sync();
      }
    }
    if (gram) {
      wg_reduce_acc<NBR>(g, lds);
      if (wave == 0) store_gram<NC>(g, gpart_of(d, s) + (int64_t)blockIdx.x * d.gpTile, n, 1.0);
    }
  };
  constexpr int KS1 = P == 2 ? 8 : 4;  // one instruction's sub-steps
  if (NCB > 1 && KS > KS1 && live_sub<P>(k) <= KS1 && n <= 16)
    run(std::integral_constant<int, 1>{}, std::integral_constant<int, (KS > KS1 ? KS1 : KS)>{});
  else
    run(std::integral_constant<int, NCB>{}, std::integral_constant<int, KS>{});
}

// ----------------------------------------------------------------------------
// Angular Galerkin reductions over directions:
//   Tm  = (sqrt(w) V)^T Qh                  r  x t   (= V^T W V-hat)
//   C   = Qh^T diag(Omega) Qh               t  x t   (= V-hat^T W Omega V-hat)
//   Ep  = Qh^T diag(1[Omega >= 0]) Qh,  En = Qh^T diag(1[Omega < 0]) Qh
//   Olo = (sqrt(w) V_lo)^T diag(1[Omega >= 0]) Qh   inflow overlap, low face
//   Ohi = (sqrt(w) V_hi)^T diag(1[Omega < 0])  Qh   inflow overlap, high face
// Partial layout (doubles): Tm @0 (ld R), C @R*T, Ep @R*T+T*T, En @R*T+2T*T,
// Olo @R*T+3T*T (ld R), Ohi @2R*T+3T*T (ld R); the t x t blocks use
// leading dimension t inside their T*T slots.
// ----------------------------------------------------------------------------
template <class S, int NCT, int NCR>
__global__ __launch_bounds__(NTHR) void k_ang_reduce(Dev d, int axis, int sd0) {
  // wavefronts 0-1 form Tm, Olo, Ohi; wavefronts 2-3 form C, Ep, En; each
  // pair walks the same strips
  constexpr int LD = 16 * (NCT + 3 * NCR) + 1;  // strip: [Qh | sw V | sw V_lo | sw V_hi]
  constexpr int NBT = NCT * (NCT + 1) / 2;
  constexpr int NRT = NCR * NCT;
  constexpr int NACC = 3 * NRT > 3 * NBT ? 3 * NRT : 3 * NBT;
  constexpr int KST = 4 * NCT, KSV = 4 * NCR;  // k-steps of 4 columns per source
  const int s = sd0 + blockIdx.y;
  const int lo = neighbour(d, s, axis, -1), hi = neighbour(d, s, axis, +1);
  const int r = d.rank[s], rl = lo >= 0 ? d.rank[lo] : 0, rh = hi >= 0 ? d.rank[hi] : 0;
  const int t = d.tdim[s];
  const int M = d.M, R = d.R, T = d.T;
  const double* om = axis == 0 ? d.omx : d.omy;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  const bool grp_v = wave < 2;
  extern __shared__ double lds[];
  double* Xs = lds + wave * (16 * LD + 16);  // strip, then 16 values of Omega
  double* oms = Xs + 16 * LD;

  const S* Qsd = (const S*)d.Qh + (int64_t)s * M * T;
  const double* Vs = d.V;
  const double* Vsrc[3] = {Vs + (int64_t)s * M * R, lo >= 0 ? Vs + (int64_t)lo * M * R : Vs,
                           hi >= 0 ? Vs + (int64_t)hi * M * R : Vs};
  const int rv[3] = {r, rl, rh};
  dbl4 acc[NACC];
  zero_acc<NACC>(acc);
  const int nst = ceil_div(M, 16);
  const int stride = gridDim.x * 2;
  // only the V-hat rows are prefetched (the three V sources would exceed the
  // register budget of the wavefronts that hold the r x t accumulators)
  S xn[KST];
  auto load = [&](int st_) {
    const int q_ = st_ * 16 + l16;
    const int qc = q_ < M ? q_ : M - 1;
#pragma unroll
    for (int ks = 0; ks < KST; ++ks) {
      const int c = 4 * ks + kq;
      const S v = Qsd[(int64_t)(c < t ? c : 0) * M + qc];
      xn[ks] = (q_ < M && c < t) ? v : (S)0;
    }
  };
  int st = blockIdx.x * 2 + (wave & 1);
  if (st < nst) load(st);
  for (; st < nst; st += stride) {
    const int q = st * 16 + l16;
    const bool rin = q < M;
    double xq[KST];
#pragma unroll
    for (int ks = 0; ks < KST; ++ks) xq[ks] = (double)xn[ks];
    if (st + stride < nst) load(st + stride);
    if (grp_v) {
      double xv[3][KSV];
#pragma unroll
      for (int b = 0; b < 3; ++b) {
#pragma unroll
        for (int ks = 0; ks < KSV; ++ks) {
          const int c = 4 * ks + kq;
          const bool in = rin && c < rv[b];
          const double v = Vsrc[b][(int64_t)(in ? c : 0) * M + (rin ? q : M - 1)];
          xv[b][ks] = in ? v : 0.0;
        }
      }
      const double swq = rin ? d.sw[q] : 0.0;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
#pragma unroll
        for (int ks = 0; ks < KSV; ++ks) Xs[l16 * LD + 16 * (NCT + b * NCR) + 4 * ks + kq] = xv[b][ks] * swq;
      }
    }
    if (kq == 0) oms[l16] = rin ? om[q] : 0.0;
#pragma unroll
    for (int ks = 0; ks < KST; ++ks) Xs[l16 * LD + 4 * ks + kq] = xq[ks];
    wave_sync();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const double o = oms[kk + kq];
      const double wp = o >= 0.0 ? 1.0 : 0.0, wn = o < 0.0 ? 1.0 : 0.0;
      const double* row = Xs + (kk + kq) * LD + l16;
      double fq[NCT];
#pragma unroll
      for (int c = 0; c < NCT; ++c) fq[c] = row[16 * c];
      if (grp_v) {
        double fo[NCR], fl[NCR], fh[NCR];
#pragma unroll
        for (int c = 0; c < NCR; ++c) {
          fo[c] = row[16 * (NCT + c)];
          fl[c] = row[16 * (NCT + NCR + c)] * wp;
          fh[c] = row[16 * (NCT + 2 * NCR + c)] * wn;
        }
#pragma unroll
        for (int a = 0; a < NCR; ++a)
#pragma unroll
          for (int b = 0; b < NCT; ++b) {
            const int i = a * NCT + b;
            acc[i] = mfma64(fo[a], fq[b], acc[i]);
            acc[NRT + i] = mfma64(fl[a], fq[b], acc[NRT + i]);
            acc[2 * NRT + i] = mfma64(fh[a], fq[b], acc[2 * NRT + i]);
          }
      } else {
        int i = 0;
#pragma unroll
        for (int bi = 0; bi < NCT; ++bi) {
#pragma unroll
          for (int bj = bi; bj < NCT; ++bj) {
            acc[i] = mfma64(fq[bi] * o, fq[bj], acc[i]);
            acc[NBT + i] = mfma64(fq[bi] * wp, fq[bj], acc[NBT + i]);
            acc[2 * NBT + i] = mfma64(fq[bi] * wn, fq[bj], acc[2 * NBT + i]);
            ++i;
          }
        }
      }
    }
    wave_sync();
  }
  pair_reduce_acc<NACC>(acc, lds);
  double* out = gpart_of(d, s) + (int64_t)blockIdx.x * d.gpTile;
  const int oC = R * T, oEp = oC + T * T, oEn = oEp + T * T, oOlo = oEn + T * T, oOhi = oOlo + R * T;
  if (wave == 0) {
#pragma unroll
    for (int a = 0; a < NCR; ++a)
#pragma unroll
      for (int b = 0; b < NCT; ++b) {
        const int i = a * NCT + b;
        store_block(out, R, r, t, a, b, acc[i], 1.0);
        store_block(out + oOlo, R, rl, t, a, b, acc[NRT + i], 1.0);
        store_block(out + oOhi, R, rh, t, a, b, acc[2 * NRT + i], 1.0);
      }
  } else if (wave == 2) {
    int i = 0;
#pragma unroll
    for (int bi = 0; bi < NCT; ++bi) {
#pragma unroll
      for (int bj = bi; bj < NCT; ++bj) {
        store_sym_block(out + oC, t, t, bi, bj, acc[i], 1.0);
        store_sym_block(out + oEp, t, t, bi, bj, acc[NBT + i], 1.0);
        store_sym_block(out + oEn, t, t, bi, bj, acc[2 * NBT + i], 1.0);
        ++i;
      }
    }
  }
}

// ----------------------------------------------------------------------------
// K-step of an advection stage (eq. advx_evolK / advy_evolK, Appendix A),
// fused with the initial value K = U (S T) and the inflow ghosts:
//   K1[p] = U[p] M0 + U[p-e] Mm + U[p+e] Mp                 (interior)
// where the missing neighbour row at the low face is replaced by
//   U[p] GLo + U_lo[its high face] GLoN,
// and at the high face by U[p] GHi + U_hi[its low face] GHiN.  The
// coefficient matrices (r x t) come from the eigen-split C = C+ + C-.
// Also leaves the partial Gram matrix K1^T K1.
// ----------------------------------------------------------------------------
template <class S, int P, int NCB, int KSP>
__global__ __launch_bounds__(NTHR) void k_kstep(Dev d, int axis, int sd0) {
  using F = typename Prec<P>::F;
  using Acc = typename Prec<P>::Acc;
  constexpr int LD = strip_ld<NCB>();
  constexpr int NB = NCB * (NCB + 1) / 2;
  // KSP: sub-steps covering the stored-rank capacity
  const int s = sd0 + blockIdx.y;
  const int lo = neighbour(d, s, axis, -1), hi = neighbour(d, s, axis, +1);
  const int r = d.rank[s], rl = lo >= 0 ? d.rank[lo] : 0, rh = hi >= 0 ? d.rank[hi] : 0;
  const int t = d.tdim[s];
  const int N = d.N, R = d.R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  extern __shared__ double lds[];
  // fragments of the 7 coefficient blocks: Cf[((m * KSP + u) * NCB + cb) * 64 + lane]
  constexpr int nfrag = 7 * KSP * NCB * 64;
  F* Cf = reinterpret_cast<F*>(lds);
  double* Ys = lds + frag_doubles<P>(nfrag) + wave * 16 * LD;
  {
    const double* sm = small_of(d, s);
    const int offs[7] = {d.oM0, d.oMm, d.oMp, d.oGLo, d.oGHi, d.oGLoN, d.oGHiN};
    const int rows[7] = {r, r, r, r, r, rl, rh};
    for (int idx = threadIdx.x; idx < nfrag; idx += NTHR) {
      const int l = idx & 63, f = idx >> 6, cb = f % NCB, u = (f / NCB) % KSP, m = f / (NCB * KSP);
      const int kc = sub_col<P>(u, l >> 4), col = 16 * cb + (l & 15);
      Cf[idx] = (kc < rows[m] && col < t) ? (F)sm[offs[m] + kc + col * R] : (F)0;
    }
  }
  __syncthreads();
  constexpr int bstride = KSP * NCB * 64;

  const double* Ub = d.U;
  const double* Us = Ub + (int64_t)s * N * R;
  const double* Ul = lo >= 0 ? Ub + (int64_t)lo * N * R : Ub;
  const double* Uh = hi >= 0 ? Ub + (int64_t)hi * N * R : Ub;
  S* K1 = (S*)d.K1 + (int64_t)s * N * d.T;
  const int e = axis == 0 ? 1 : d.lnx;
  const int na = axis == 0 ? d.lnx : d.lny;
  dbl4 g[NB];
  zero_acc<NB>(g);
  const int nst = ceil_div(N, 16);
  const int stride = gridDim.x * NW;
  F n0[KSP], nm[KSP], np[KSP];
  auto load = [&](int st_) {
    const int p_ = st_ * 16 + l16;
    const bool rin_ = p_ < N;
    const int pc = rin_ ? p_ : N - 1;
    const int ia_ = axis == 0 ? pc % d.lnx : pc / d.lnx;
    const bool hm_ = rin_ && ia_ > 0, hp_ = rin_ && ia_ < na - 1;
    const int pm_ = hm_ ? pc - e : pc, pp_ = hp_ ? pc + e : pc;
#pragma unroll
    for (int u = 0; u < KSP; ++u) {
      const int kc = sub_col<P>(u, kq);
      const bool kin = kc < r;
      const int64_t col = (int64_t)(kin ? kc : 0) * N;
      const double v0 = Us[col + pc], vm = Us[col + pm_], vp = Us[col + pp_];
      n0[u] = (rin_ && kin) ? (F)v0 : (F)0;
      nm[u] = (hm_ && kin) ? (F)vm : (F)0;
      np[u] = (hp_ && kin) ? (F)vp : (F)0;
    }
  };
  int st = blockIdx.x * NW + wave;
  if (st < nst) load(st);
  for (; st < nst; st += stride) {
    const int p = st * 16 + l16;
    const bool rin = p < N;
    const int ix = p % d.lnx, iy = p / d.lnx;
    const int ia = axis == 0 ? ix : iy;
    const int f = axis == 0 ? iy : ix;
    const bool flo = rin && ia == 0, fhi = rin && ia == na - 1;
    F u0[KSP], um[KSP], up[KSP];
#pragma unroll
    for (int u = 0; u < KSP; ++u) {
      u0[u] = n0[u];
      um[u] = nm[u];
      up[u] = np[u];
    }
    if (st + stride < nst) load(st + stride);
    Acc acc[NCB];
    zero_prod<P>(acc, NCB);
    prod_acc<P, NCB, KSP>(acc, Cf, u0);
    prod_acc<P, NCB, KSP>(acc, Cf + bstride, um);
    prod_acc<P, NCB, KSP>(acc, Cf + 2 * bstride, up);
    if (__any(flo)) {
      const int pn = face_cell(d, axis, true, f);
      F gu[KSP], gn[KSP];
#pragma unroll
      for (int u = 0; u < KSP; ++u) {
        const int kc = sub_col<P>(u, kq);
        gu[u] = flo ? u0[u] : (F)0;
        const bool in = flo && lo >= 0 && kc < rl;
        const double v = Ul[(int64_t)(in ? kc : 0) * N + pn];
        gn[u] = in ? (F)v : (F)0;
      }
      prod_acc<P, NCB, KSP>(acc, Cf + 3 * bstride, gu);
      prod_acc<P, NCB, KSP>(acc, Cf + 5 * bstride, gn);
    }
    if (__any(fhi)) {
      const int pn = face_cell(d, axis, false, f);
      F gu[KSP], gn[KSP];
#pragma unroll
      for (int u = 0; u < KSP; ++u) {
        const int kc = sub_col<P>(u, kq);
        gu[u] = fhi ? u0[u] : (F)0;
        const bool in = fhi && hi >= 0 && kc < rh;
        const double v = Uh[(int64_t)(in ? kc : 0) * N + pn];
        gn[u] = in ? (F)v : (F)0;
      }
      prod_acc<P, NCB, KSP>(acc, Cf + 4 * bstride, gu);
      prod_acc<P, NCB, KSP>(acc, Cf + 6 * bstride, gn);
    }
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = out_col<P>(cb, v, kq);
        const S val = rin ? (S)acc[cb][v] : (S)0;
        if (rin && j < t) K1[(int64_t)j * N + p] = val;
        Ys[l16 * LD + j] = (double)val;
      }
    }
    wave_sync();
    strip_gram<NCB, LD>(g, Ys);
    wave_sync();
  }
  wg_reduce_acc<NB>(g, lds);
  if (wave == 0) store_gram<NCB>(g, gpart_of(d, s) + (int64_t)blockIdx.x * d.gpTile, t, 1.0);
}

// ----------------------------------------------------------------------------
// Spatial Galerkin matrices of the S- and L-steps (eqs. advx_evolS/L):
//   Gm[i,j] = sum_p Q[p,i] (Q[p,j] - Q[p-e,j])   (zero beyond the low face)
//   Gp[i,j] = sum_p Q[p,i] (Q[p+e,j] - Q[p,j])   (zero beyond the high face)
// with Q = h U^1.  Both follow from one product: with
//   B[i,j] = sum_{p not on the high face} Q[p,i] Q[p+e,j]  and  C = Q^T Q,
// shifting p by e shows sum_{p not on the low face} Q[p,i] Q[p-e,j] =
// B[j,i], so Gp = B - C and Gm = C - B^T = -Gp^T (C is symmetric).  Gp is
// formed as sum_p Q[p,i] (Q[p+e,j] - Q[p,j]) with the difference taken per
// element in FP64 (exact for stored values, no cancellation between B and
// C), and the S-step kernel sets Gm = -Gp^T.
// Also the face products of the frozen inflow data (t x r blocks):
//   Xlo = Q[lo face]^T U[lo face],   Xln = Q[lo face]^T U_lo[its hi face],
//   Xhi = Q[hi face]^T U[hi face],   Xhn = Q[hi face]^T U_hi[its lo face].
// Gp: every wavefront walks its own strips of cells; the face products run
// over the face cells gathered into strips of 16 (items dealt to the
// wavefronts of all workgroups).  Partial layout: Gp @0 (t x t, ld t),
// Xlo @2T*T, Xhi @2T*T+T*R, Xln @2T*T+2T*R, Xhn @2T*T+3T*R (t x r_*, ld T).
// ----------------------------------------------------------------------------
template <class S, int NCT, int NCR>
__global__ __launch_bounds__(NTHR) void k_spatial_reduce(Dev d, int axis, int sd0, const void* Q) {
  // Operands are loaded straight into the matrix-core lane layout (lane:
  // column 16 c + l mod 16 of Q, row 4 k + l / 16 of the strip): a strip of
  // 16 rows reads 16 columns x 16 rows, whole cache lines, with no LDS
  // transposition.
  constexpr int NQ = NCT * NCT;
  constexpr int NX = NCT * NCR;
  const int s = sd0 + blockIdx.y;
  const int t = d.tdim[s];
  const int N = d.N, T = d.T, R = d.R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  extern __shared__ double lds[];
  const S* Qsd = (const S*)Q + (int64_t)s * N * T;
  const int e = axis == 0 ? 1 : d.lnx;
  const int na = axis == 0 ? d.lnx : d.lny;
  double* out = gpart_of(d, s) + (int64_t)blockIdx.x * d.gpTile;
  const int lo = neighbour(d, s, axis, -1), hi = neighbour(d, s, axis, +1);
  const int r = d.rank[s], rl = lo >= 0 ? d.rank[lo] : 0, rh = hi >= 0 ? d.rank[hi] : 0;
  const double* Us = d.U + (int64_t)s * N * R;
  dbl4 acc[NQ + 4 * NX];  // Gp, then Xlo, Xln, Xhi, Xhn
  zero_acc<NQ + 4 * NX>(acc);
  const int nst = ceil_div(N, 16);
  const int stride = gridDim.x * NW;
  S a0[4][NCT], a1[4][NCT];  // Q and Q shifted by +e, k steps x column blocks
  auto load = [&](int st_) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int p_ = st_ * 16 + 4 * kk + kq;
      const bool rin_ = p_ < N;
      const int ia_ = axis == 0 ? p_ % d.lnx : p_ / d.lnx;
      const bool hs_ = rin_ && ia_ < na - 1;  // p + e inside the subdomain
      const int pr = rin_ ? p_ : 0, ps = hs_ ? p_ + e : 0;
#pragma unroll
      for (int c = 0; c < NCT; ++c) {
        const int col = 16 * c + l16;
        const int cc = col < t ? col : 0;
        const S v0 = Qsd[(int64_t)cc * N + pr];
        const S v1 = Qsd[(int64_t)cc * N + ps];
        a0[kk][c] = (rin_ && col < t) ? v0 : (S)0;
        a1[kk][c] = (hs_ && col < t) ? v1 : (S)0;
      }
    }
  };
  int st = blockIdx.x * NW + wave;
  if (st < nst) load(st);
  // face products over the face cells, gathered into strips of 16: items
  // (side, strip) dealt to the wavefronts of all workgroups, done while the
  // first strip of Gp is in flight
  const int flen = face_len(d, axis), nfs = ceil_div(flen, 16);
  for (int item = blockIdx.x * NW + wave; item < 2 * nfs; item += stride) {
    const int side = item / nfs;  // 0 low, 1 high (wave-uniform)
    const int nb = side == 0 ? lo : hi;
    const int rn = side == 0 ? rl : rh;
    const double* Unb = nb >= 0 ? d.U + (int64_t)nb * N * R : d.U;
    double q[4][NCT], uo[4][NCR], un[4][NCR];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int fcell = (item % nfs) * 16 + 4 * kk + kq;
      const bool ok = fcell < flen;
      const int p = face_cell(d, axis, side == 1, ok ? fcell : 0);
      const int pf = face_cell(d, axis, side == 0, ok ? fcell : 0);  // the neighbour's touching cell
#pragma unroll
      for (int c = 0; c < NCT; ++c) {
        const int col = 16 * c + l16;
        q[kk][c] = (ok && col < t) ? (double)Qsd[(int64_t)col * N + p] : 0.0;
      }
#pragma unroll
      for (int c = 0; c < NCR; ++c) {
        const int col = 16 * c + l16;
        uo[kk][c] = (ok && col < r) ? Us[(int64_t)col * N + p] : 0.0;
        un[kk][c] = (ok && col < rn) ? Unb[(int64_t)col * N + pf] : 0.0;
      }
    }
    if (side == 0) {
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int bi = 0; bi < NCT; ++bi)
#pragma unroll
          for (int bc = 0; bc < NCR; ++bc) {
            acc[NQ + bi * NCR + bc] = mfma64(q[kk][bi], uo[kk][bc], acc[NQ + bi * NCR + bc]);
            acc[NQ + NX + bi * NCR + bc] = mfma64(q[kk][bi], un[kk][bc], acc[NQ + NX + bi * NCR + bc]);
          }
    } else {
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int bi = 0; bi < NCT; ++bi)
#pragma unroll
          for (int bc = 0; bc < NCR; ++bc) {
            acc[NQ + 2 * NX + bi * NCR + bc] = mfma64(q[kk][bi], uo[kk][bc], acc[NQ + 2 * NX + bi * NCR + bc]);
            acc[NQ + 3 * NX + bi * NCR + bc] = mfma64(q[kk][bi], un[kk][bc], acc[NQ + 3 * NX + bi * NCR + bc]);
          }
    }
  }
  // Gp over all strips, every wavefront on its own strips
  for (; st < nst; st += stride) {
    double x0[4][NCT], x1[4][NCT];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int c = 0; c < NCT; ++c) {
        x0[kk][c] = (double)a0[kk][c];
        x1[kk][c] = (double)a1[kk][c];
      }
    if (st + stride < nst) load(st + stride);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int bi = 0; bi < NCT; ++bi)
#pragma unroll
        for (int bj = 0; bj < NCT; ++bj)
          acc[bi * NCT + bj] = mfma64(x0[kk][bi], x1[kk][bj] - x0[kk][bj], acc[bi * NCT + bj]);
  }
  wg_reduce_acc<NQ + 4 * NX>(acc, lds);
  if (wave == 0) {
#pragma unroll
    for (int bi = 0; bi < NCT; ++bi) {
#pragma unroll
      for (int bj = 0; bj < NCT; ++bj) store_block(out, t, t, t, bi, bj, acc[bi * NCT + bj], 1.0);
#pragma unroll
      for (int bc = 0; bc < NCR; ++bc) {
        store_block(out + 2 * T * T, T, t, r, bi, bc, acc[NQ + bi * NCR + bc], 1.0);
        store_block(out + 2 * T * T + 2 * T * R, T, t, rl, bi, bc, acc[NQ + NX + bi * NCR + bc], 1.0);
        store_block(out + 2 * T * T + T * R, T, t, r, bi, bc, acc[NQ + 2 * NX + bi * NCR + bc], 1.0);
        store_block(out + 2 * T * T + 3 * T * R, T, t, rh, bi, bc, acc[NQ + 3 * NX + bi * NCR + bc], 1.0);
      }
    }
  }
}

// ----------------------------------------------------------------------------
// L-step of an advection stage (eq. advx_evolL), weighted by sqrt(w):
//   AL[q,:] = Qh[q,:] (P0 + Omega_q^+ Pm + Omega_q^- Pp)
// with P0 = S2^T, Pm = -dt c Hm^T, Pp = -dt c Hp^T; each direction is
// upwinded by the sign of its own Omega.  Leaves the partial Gram of AL.
// ----------------------------------------------------------------------------
template <class S, int P, int NCB, int KS>
__global__ __launch_bounds__(NTHR) void k_lstep(Dev d, int axis, int sd0) {
  using F = typename Prec<P>::F;
  using Acc = typename Prec<P>::Acc;
  constexpr int LD = strip_ld<NCB>();
  constexpr int NB = NCB * (NCB + 1) / 2;
  const int s = sd0 + blockIdx.y;
  const int t = d.tdim[s];
  const int M = d.M, T = d.T;
  const double* om = axis == 0 ? d.omx : d.omy;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  extern __shared__ double lds[];
  // fragments of P0, Pm, Pp: Pf[((m * KS + u) * NCB + cb) * 64 + lane]
  constexpr int nfrag = 3 * KS * NCB * 64;
  F* Pf = reinterpret_cast<F*>(lds);
  double* Ys = lds + frag_doubles<P>(nfrag) + wave * 16 * LD;
  {
    const double* sm = small_of(d, s);
    const int offs[3] = {d.oP0, d.oPm, d.oPp};
    for (int idx = threadIdx.x; idx < nfrag; idx += NTHR) {
      const int l = idx & 63, f = idx >> 6, cb = f % NCB, u = (f / NCB) % KS, m = f / (NCB * KS);
      const int kc = sub_col<P>(u, l >> 4), col = 16 * cb + (l & 15);
      Pf[idx] = (kc < t && col < t) ? (F)sm[offs[m] + kc + col * T] : (F)0;
    }
  }
  __syncthreads();
  constexpr int bstride = KS * NCB * 64;
  const S* Qsd = (const S*)d.Qh + (int64_t)s * M * T;
  S* ALs = (S*)d.AL + (int64_t)s * M * T;
  dbl4 g[NB];
  zero_acc<NB>(g);
  const int nst = ceil_div(M, 16);
  const int stride = gridDim.x * NW;
  F xn[KS];
  double on_ = 0.0;
  auto load = [&](int st_) {
    const int q_ = st_ * 16 + l16;
    const int qc = q_ < M ? q_ : M - 1;
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      const int kc = sub_col<P>(u, kq);
      const bool in = q_ < M && kc < t;
      const S v = Qsd[(int64_t)(in ? kc : 0) * M + qc];
      xn[u] = in ? (F)v : (F)0;
    }
    const double o_ = om[qc];
    on_ = q_ < M ? o_ : 0.0;
  };
  int st = blockIdx.x * NW + wave;
  if (st < nst) load(st);
  for (; st < nst; st += stride) {
    const int q = st * 16 + l16;
    const bool rin = q < M;
    const double o = on_;
    const F op = (F)(o >= 0.0 ? o : 0.0), on = (F)(o < 0.0 ? o : 0.0);
    F xv[KS], xm[KS], xp[KS];
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      xv[u] = xn[u];
      xm[u] = xv[u] * op;
      xp[u] = xv[u] * on;
    }
    if (st + stride < nst) load(st + stride);
    Acc acc[NCB];
    zero_prod<P>(acc, NCB);
    prod_acc<P, NCB, KS>(acc, Pf, xv);
    prod_acc<P, NCB, KS>(acc, Pf + bstride, xm);
    prod_acc<P, NCB, KS>(acc, Pf + 2 * bstride, xp);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = out_col<P>(cb, v, kq);
        const S val = rin ? (S)acc[cb][v] : (S)0;
        if (rin && j < t) ALs[(int64_t)j * M + q] = val;
        Ys[l16 * LD + j] = (double)val;
      }
    }
    wave_sync();
    strip_gram<NCB, LD>(g, Ys);
    wave_sync();
  }
  wg_reduce_acc<NB>(g, lds);
  if (wave == 0) store_gram<NCB>(g, gpart_of(d, s) + (int64_t)blockIdx.x * d.gpTile, t, 1.0);
}

// ----------------------------------------------------------------------------
// Collision stage K-step (eq. coll_evolK), K = U S, m = V^T w:
//   K1[p] = (1 - dt c_t[p]) K[p] + dt (c_s[p]/W) (K[p].m) m + dt Q[p] m
// formed from one product U [S | S m], whose last column is K[p].m.  Leaves
// the partial Gram of K1 (r columns).
// ----------------------------------------------------------------------------
template <class S, int P, int NCB, int KSP>
__global__ __launch_bounds__(NTHR) void k_coll_kstep(Dev d, int sd0) {
  using F = typename Prec<P>::F;
  using Acc = typename Prec<P>::Acc;
  constexpr int LD = strip_ld<NCB>();
  constexpr int NB = NCB * (NCB + 1) / 2;
  // KSP: sub-steps covering the stored-rank capacity
  const int s = sd0 + blockIdx.y;
  const int r = d.rank[s];
  const int N = d.N, R = d.R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  __shared__ double Bs[CAPR * (CAPR + 1)];  // [S | S m], leading dimension CAPR
  __shared__ double mv[16 * NCB];
  __shared__ F Bf[KSP * NCB * 64];
  __shared__ double Ysh[NW * 16 * LD];
  double* Ys = Ysh + wave * 16 * LD;
  const double* sm = small_of(d, s);
  const double* Sg = d.S + (int64_t)s * R * R;
  for (int idx = threadIdx.x; idx < r * r; idx += NTHR) {
    const int a = idx % r, b = idx / r;
    Bs[a + b * CAPR] = Sg[a + b * R];
  }
  for (int a = threadIdx.x; a < 16 * NCB; a += NTHR) mv[a] = a < r ? sm[d.oMv + a] : 0.0;
  __syncthreads();
  for (int a = threadIdx.x; a < r; a += NTHR) {
    double acc = 0.0;
    for (int b = 0; b < r; ++b) acc = fma(Bs[a + b * CAPR], mv[b], acc);
    Bs[a + r * CAPR] = acc;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < KSP * NCB * 64; idx += NTHR) {
    const int l = idx & 63, f = idx >> 6, cb = f % NCB, u = f / NCB;
    const int kc = sub_col<P>(u, l >> 4), col = 16 * cb + (l & 15);
    Bf[idx] = (kc < r && col <= r) ? (F)Bs[kc + col * CAPR] : (F)0;
  }
  __syncthreads();

  const double* Us = d.U + (int64_t)s * N * R;
  const double* cs = d.cs + (int64_t)s * N;
  const double* ct = d.ct + (int64_t)s * N;
  const double* Qs = d.Qsrc + (int64_t)s * N;
  S* K1 = (S*)d.K1 + (int64_t)s * N * d.T;
  const double dt = d.dt, iW = 1.0 / d.W;
  const int src_lane = l16 + 16 * out_kq<P>(r);  // lane holding column r of this row
  dbl4 g[NB];
  zero_acc<NB>(g);
  const int nst = ceil_div(N, 16);
  const int stride = gridDim.x * NW;
  F xn[KSP];
  double ctn = 0.0, csn = 0.0, qn = 0.0;
  auto load = [&](int st_) {
    const int p_ = st_ * 16 + l16;
    const bool rin_ = p_ < N;
    const int pc = rin_ ? p_ : N - 1;
#pragma unroll
    for (int u = 0; u < KSP; ++u) {
      const int kc = sub_col<P>(u, kq);
      const bool in = rin_ && kc < r;
      const double v = Us[(int64_t)(in ? kc : 0) * N + pc];
      xn[u] = in ? (F)v : (F)0;
    }
    const double a = ct[pc], b = cs[pc], c = Qs[pc];
    ctn = rin_ ? a : 0.0;
    csn = rin_ ? b : 0.0;
    qn = rin_ ? c : 0.0;
  };
  int st = blockIdx.x * NW + wave;
  if (st < nst) load(st);
  for (; st < nst; st += stride) {
    const int p = st * 16 + l16;
    const bool rin = p < N;
    F xv[KSP];
#pragma unroll
    for (int u = 0; u < KSP; ++u) xv[u] = xn[u];
    const double ctp = ctn, csp = csn, qp = qn;
    if (st + stride < nst) load(st + stride);
    Acc acc[NCB];
    zero_prod<P>(acc, NCB);
    prod_acc<P, NCB, KSP>(acc, Bf, xv);
    double kmv = 0.0;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (out_col<P>(cb, v, kq) == r) kmv = (double)acc[cb][v];
    const double km = __shfl(kmv, src_lane, 64);
    const double a0 = rin ? 1.0 - dt * ctp : 0.0;
    const double a1 = rin ? dt * (csp * iW * km + qp) : 0.0;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = out_col<P>(cb, v, kq);
        const S val = (rin && j < r) ? (S)fma(a0, (double)acc[cb][v], a1 * mv[j]) : (S)0;
        if (rin && j < r) K1[(int64_t)j * N + p] = val;
        Ys[l16 * LD + j] = (double)val;
      }
    }
    wave_sync();
    strip_gram<NCB, LD>(g, Ys);
    wave_sync();
  }
  wg_reduce_acc<NB>(g, Ysh);
  if (wave == 0) store_gram<NCB>(g, gpart_of(d, s) + (int64_t)blockIdx.x * d.gpTile, r, 1.0);
}

// ----------------------------------------------------------------------------
// Collision Galerkin reductions (eq. coll_evolS/L) from U^1 (already in the
// state buffer):  Gs = h^2 U^T diag(c_s) U,  Gt = h^2 U^T diag(c_t) U,
// qv = h^2 U^T Q.  Partial layout: Gs @0, Gt @R*R (ld R), qv @2R*R.
// ----------------------------------------------------------------------------
template <int NCB>
__global__ __launch_bounds__(NTHR) void k_coll_reduce(Dev d, int sd0) {
  constexpr int LD = strip_ld<NCB>();
  constexpr int NB = NCB * (NCB + 1) / 2;
  constexpr int NACC = 2 * NB + NCB;
  constexpr int KS = 4 * NCB;
  const int s = sd0 + blockIdx.y;
  const int r = d.rank[s];
  const int N = d.N, R = d.R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  __shared__ double sh[NW * (16 * LD + 48)];
  __shared__ double red[NACC * 256];
  double* Us = sh + wave * (16 * LD + 48);  // strip, then c_s, c_t, Q of its rows
  double* wv = Us + 16 * LD;
  const double* Ug = d.U + (int64_t)s * N * R;
  const double* cs = d.cs + (int64_t)s * N;
  const double* ct = d.ct + (int64_t)s * N;
  const double* Qg = d.Qsrc + (int64_t)s * N;
  dbl4 acc[NACC];
  zero_acc<NACC>(acc);
  const int nst = ceil_div(N, 16);
  const int stride = gridDim.x * NW;
  double xn[KS];
  double wn = 0.0;
  auto load = [&](int st_) {
    const int p_ = st_ * 16 + l16;
    const bool rin_ = p_ < N;
    const int pc = rin_ ? p_ : N - 1;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int c = 4 * ks + kq;
      const bool in = rin_ && c < r;
      const double v = Ug[(int64_t)(in ? c : 0) * N + pc];
      xn[ks] = in ? v : 0.0;
    }
    // three plain loads and a select: a pointer chosen per lane would be
    // kept in a private array (scratch) by the compiler
    const double w0 = cs[pc], w1 = ct[pc], w2 = Qg[pc];
    const double w_ = kq == 0 ? w0 : (kq == 1 ? w1 : w2);
    wn = (rin_ && kq < 3) ? w_ : 0.0;
  };
  int st = blockIdx.x * NW + wave;
  if (st < nst) load(st);
  for (; st < nst; st += stride) {
    double xv[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) xv[ks] = xn[ks];
    const double wsrc = wn;
    if (st + stride < nst) load(st + stride);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) Us[l16 * LD + 4 * ks + kq] = xv[ks];
    if (kq < 3) wv[kq * 16 + l16] = wsrc;
    wave_sync();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const int row = kk + kq;
      const double ws = wv[row], wt = wv[16 + row], wq = wv[32 + row];
      double f[NCB];
#pragma unroll
      for (int c = 0; c < NCB; ++c) f[c] = Us[row * LD + 16 * c + l16];
      int idx = 0;
#pragma unroll
      for (int bi = 0; bi < NCB; ++bi) {
#pragma unroll
        for (int bj = bi; bj < NCB; ++bj) {
          acc[idx] = mfma64(f[bi] * ws, f[bj], acc[idx]);
          acc[idx + NB] = mfma64(f[bi] * wt, f[bj], acc[idx + NB]);
          ++idx;
        }
      }
      const double bq = l16 == 0 ? wq : 0.0;
#pragma unroll
      for (int c = 0; c < NCB; ++c) acc[2 * NB + c] = mfma64(f[c], bq, acc[2 * NB + c]);
    }
    wave_sync();
  }
  wg_reduce_acc<NACC>(acc, red);
  if (wave == 0) {
    double* out = gpart_of(d, s) + (int64_t)blockIdx.x * d.gpTile;
    const double h2 = d.h * d.h;
    int idx = 0;
#pragma unroll
    for (int bi = 0; bi < NCB; ++bi) {
#pragma unroll
      for (int bj = bi; bj < NCB; ++bj) {
        store_sym_block(out, R, r, bi, bj, acc[idx], h2);
        store_sym_block(out + R * R, R, r, bi, bj, acc[idx + NB], h2);
        ++idx;
      }
    }
#pragma unroll
    for (int c = 0; c < NCB; ++c) store_block(out + 2 * R * R, 1, r, 1, c, 0, acc[2 * NB + c], h2);
  }
}

// ----------------------------------------------------------------------------
// Collision L-step (eq. coll_evolL), weighted by sqrt(w):
//   AL[q,:] = sqrt(w_q) (V[q,:] P + crow),  P = S2^T (I - dt Gt),
//   crow = dt ((S2 m)^T Gs / W + q^T).  Leaves the partial Gram of AL.
// ----------------------------------------------------------------------------
template <class S, int P, int NCB, int KSP>
__global__ __launch_bounds__(NTHR) void k_coll_lstep(Dev d, int sd0) {
  using F = typename Prec<P>::F;
  using Acc = typename Prec<P>::Acc;
  constexpr int LD = strip_ld<NCB>();
  const int s = sd0 + blockIdx.y;
  const int r = d.rank[s];
  const int M = d.M, R = d.R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  __shared__ double cr[16 * NCB];
  __shared__ F Bf[KSP * NCB * 64];
  __shared__ double Ysh[NW * 16 * LD];
  double* Ys = Ysh + wave * 16 * LD;
  const double* sm = small_of(d, s);
  for (int idx = threadIdx.x; idx < KSP * NCB * 64; idx += NTHR) {
    const int l = idx & 63, f = idx >> 6, cb = f % NCB, u = f / NCB;
    const int kc = sub_col<P>(u, l >> 4), col = 16 * cb + (l & 15);
    Bf[idx] = (kc < r && col < r) ? (F)sm[d.oP0 + kc + col * R] : (F)0;
  }
  for (int a = threadIdx.x; a < 16 * NCB; a += NTHR) cr[a] = a < r ? sm[d.oCrow + a] : 0.0;
  __syncthreads();
  const double* Vs = d.V + (int64_t)s * M * R;
  S* ALs = (S*)d.AL + (int64_t)s * M * d.T;
  const int nst = ceil_div(M, 16);
  const int stride = gridDim.x * NW;
  // NC output column blocks and KSR sub-steps are issued: a subdomain of
  // rank at most one instruction's columns (and 16) takes the short instance
  auto run = [&](auto nc_c, auto ks_c) {
    constexpr int NC = decltype(nc_c)::value, KSR = decltype(ks_c)::value;
    constexpr int NBR = NC * (NC + 1) / 2;
    dbl4 g[NBR];
    zero_acc<NBR>(g);
    F xn[KSR];
    double swn = 0.0;
    auto load = [&](int st_) {
      const int q_ = st_ * 16 + l16;
      const int qc = q_ < M ? q_ : M - 1;
#pragma unroll
      for (int u = 0; u < KSR; ++u) {
        const int kc = sub_col<P>(u, kq);
        const bool in = q_ < M && kc < r;
        const double v = Vs[(int64_t)(in ? kc : 0) * M + qc];
        xn[u] = in ? (F)v : (F)0;
      }
      const double w_ = d.sw[qc];
      swn = q_ < M ? w_ : 0.0;
    };
    int st = blockIdx.x * NW + wave;
    if (st < nst) load(st);
    for (; st < nst; st += stride) {
      const int q = st * 16 + l16;
      const bool rin = q < M;
      F xv[KSR];
#pragma unroll
      for (int u = 0; u < KSR; ++u) xv[u] = xn[u];
      const double swq = swn;
      if (st + stride < nst) load(st + stride);
      Acc acc[NC];
      zero_prod<P>(acc, NC);
      prod_acc<P, NC, KSR, NCB>(acc, Bf, xv);
#pragma unroll
      for (int cb = 0; cb < NC; ++cb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = out_col<P>(cb, v, kq);
          const S val = (rin && j < r) ? (S)(swq * ((double)acc[cb][v] + cr[j])) : (S)0;
          if (rin && j < r) ALs[(int64_t)j * M + q] = val;
          Ys[l16 * LD + j] = (double)val;
        }
      }
      wave_sync();
      strip_gram<NC, LD>(g, Ys);
      wave_sync();
    }
    wg_reduce_acc<NBR>(g, Ysh);
    if (wave == 0) store_gram<NC>(g, gpart_of(d, s) + (int64_t)blockIdx.x * d.gpTile, r, 1.0);
  };
  constexpr int KS1 = P == 2 ? 8 : 4;  // one instruction's sub-steps
  if (NCB > 1 && KSP > KS1 && live_sub<P>(r) <= KS1 && r <= 16)
    run(std::integral_constant<int, 1>{}, std::integral_constant<int, (KSP > KS1 ? KS1 : KSP)>{});
  else
    run(std::integral_constant<int, NCB>{}, std::integral_constant<int, KSP>{});
}

// ----------------------------------------------------------------------------
// Angular moments on the global grid: scalar flux rho = U (S (V^T w)) (Section
// 2) and current density jx = U (S (V^T (w Omega_x))), jy likewise; written to
// d.rho, d.rho + nx ny and d.rho + 2 nx ny.  nmom = 1 forms rho only.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(NTHR) void k_moments(Dev d, int nmom) {
  const int s = blockIdx.y;
  const int r = d.rank[s];
  const int N = d.N, M = d.M, R = d.R;
  constexpr int MV = 64;  // largest stored rank of either plan
  __shared__ double mv[3 * MV];
  __shared__ double smv[3 * MV];
  const double* Vs = d.V + (int64_t)s * M * R;
  // (V^T (w Omega_m))_a for a < r, m < nmom (Omega_0 = 1), one per thread in
  // a fixed order over the directions
  for (int idx = threadIdx.x; idx < nmom * r; idx += NTHR) {
    const int a = idx % r, m = idx / r;
    const double* om = m == 1 ? d.omx : d.omy;
    double acc = 0.0;
    for (int q = 0; q < M; ++q) {
      const double wq = m == 0 ? d.w[q] : d.w[q] * om[q];
      acc = fma(Vs[(int64_t)a * M + q], wq, acc);
    }
    mv[m * MV + a] = acc;
  }
  __syncthreads();
  const double* Sg = d.S + (int64_t)s * R * R;
  for (int idx = threadIdx.x; idx < nmom * r; idx += NTHR) {
    const int a = idx % r, m = idx / r;
    double acc = 0.0;
    for (int b = 0; b < r; ++b) acc = fma(Sg[a + b * R], mv[m * MV + b], acc);
    smv[m * MV + a] = acc;
  }
  __syncthreads();
  const double* Us = d.U + (int64_t)s * N * R;
  const int sx = s % d.px, sy = s / d.px;
  const int64_t plane = (int64_t)d.nx * d.lny * d.py;  // cells of the global grid
  for (int p = blockIdx.x * NTHR + threadIdx.x; p < N; p += gridDim.x * NTHR) {
    const int ix = p % d.lnx, iy = p / d.lnx;
    const int64_t g = (int64_t)(sy * d.lny + iy) * d.nx + sx * d.lnx + ix;
    for (int m = 0; m < nmom; ++m) {
      double acc = 0.0;
      for (int a = 0; a < r; ++a) acc = fma(Us[(int64_t)a * N + p], smv[m * MV + a], acc);
      d.rho[m * plane + g] = acc;
    }
  }
}

// The same moments in two launches with the per-subdomain vectors in a
// caller-provided buffer (no staging on the global grid): k_moments_vec
// forms smv[s][m][a] = (S (V^T (w Omega_m)))_a, k_moments_apply writes the
// moments of every cell straight to the destinations.  The arithmetic (and
// its order) is that of k_moments, so the results are identical.
__global__ __launch_bounds__(NTHR) void k_moments_vec(Dev d, int nmom, double* smv_out) {
  const int s = blockIdx.x;
  const int r = d.rank[s];
  const int M = d.M, R = d.R;
  constexpr int MV = 64;
  __shared__ double mv[3 * MV];
  const double* Vs = d.V + (int64_t)s * M * R;
  for (int idx = threadIdx.x; idx < nmom * r; idx += NTHR) {
    const int a = idx % r, m = idx / r;
    const double* om = m == 1 ? d.omx : d.omy;
    double acc = 0.0;
    for (int q = 0; q < M; ++q) {
      const double wq = m == 0 ? d.w[q] : d.w[q] * om[q];
      acc = fma(Vs[(int64_t)a * M + q], wq, acc);
    }
    mv[m * MV + a] = acc;
  }
  __syncthreads();
  const double* Sg = d.S + (int64_t)s * R * R;
  for (int idx = threadIdx.x; idx < nmom * r; idx += NTHR) {
    const int a = idx % r, m = idx / r;
    double acc = 0.0;
    for (int b = 0; b < r; ++b) acc = fma(Sg[a + b * R], mv[m * MV + b], acc);
    smv_out[((int64_t)s * 3 + m) * MV + a] = acc;
  }
}

__global__ __launch_bounds__(NTHR) void k_moments_apply(Dev d, int nmom, const double* smv, double* rho, double* jx,
                                                        double* jy) {
  const int s = blockIdx.y;
  const int r = d.rank[s];
  const int N = d.N, R = d.R;
  constexpr int MV = 64;
  const double* Us = d.U + (int64_t)s * N * R;
  const double* sv = smv + (int64_t)s * 3 * MV;
  const int sx = s % d.px, sy = s / d.px;
  double* dst[3] = {rho, jx, jy};
  for (int p = blockIdx.x * NTHR + threadIdx.x; p < N; p += gridDim.x * NTHR) {
    const int ix = p % d.lnx, iy = p / d.lnx;
    const int64_t g = (int64_t)(sy * d.lny + iy) * d.nx + sx * d.lnx + ix;
    for (int m = 0; m < nmom; ++m) {
      double acc = 0.0;
      for (int a = 0; a < r; ++a) acc = fma(Us[(int64_t)a * N + p], sv[m * MV + a], acc);
      dst[m][g] = acc;
    }
  }
}

// ============================================================================
// Host-side launchers: pick the template instance from the precision mode and
// the capacities.
// ============================================================================
namespace {

template <int V>
using ic = std::integral_constant<int, V>;
template <class T>
struct tag {
  using type = T;
};

// column blocks of 16 covering a capacity of n columns (1..4)
int ncb_of(int n) { return n <= 16 ? 1 : (n <= 32 ? 2 : (n <= 48 ? 3 : 4)); }

template <class Fn>
void with_ncb(int ncb, Fn f) {
  switch (ncb) {
    case 1: f(ic<1>{}); break;
    case 2: f(ic<2>{}); break;
    case 3: f(ic<3>{}); break;
    default: f(ic<4>{}); break;
  }
}

// storage type and product precision of a launch: FP64 mode stores and
// computes in FP64; the mixed modes store in FP32 and compute products in
// FP32 or split BF16, except QR products (exact), which stay FP64
template <class Fn>
void with_prec(int prec, bool exact, Fn f) {
  if (prec == DD_PREC_FP64) f(tag<double>{}, ic<0>{});
  else if (exact) f(tag<float>{}, ic<0>{});
  else if (prec == DD_PREC_MIXED_FP32) f(tag<float>{}, ic<1>{});
  else f(tag<float>{}, ic<2>{});
}

template <class Fn>
void with_store(int prec, Fn f) {
  if (prec == DD_PREC_FP64) f(tag<double>{});
  else f(tag<float>{});
}

// sub-steps of the coefficient fragments for a capacity of n rows
int sub_steps(int P, int n) { return P == 2 ? 8 * ceil_div(n, 32) : ceil_div(n, 4); }

// compile-time sub-step count covering the stored-rank capacity (at most
// CAPR = 21 ranks: six 4-column sub-steps, or one 32-column BF16 group)
template <int P, class Fn>
void with_ksp(int rcap, Fn f) {
  if constexpr (P == 2) {
    f(ic<8>{});
  } else {
    switch (ceil_div(rcap, 4)) {
      case 1: f(ic<1>{}); break;
      case 2: f(ic<2>{}); break;
      case 3: f(ic<3>{}); break;
      case 4: f(ic<4>{}); break;
      case 5: f(ic<5>{}); break;
      default: f(ic<6>{}); break;
    }
  }
}

constexpr size_t D8 = sizeof(double);

// dynamic LDS of the row reductions (one helper for the launch and for the
// occupancy query)
template <int NT, int NR>
constexpr size_t ang_reduce_lds() {
  constexpr int NACC = std::max(3 * NR * NT, 3 * NT * (NT + 1) / 2);
  return D8 * std::max<size_t>(NW * (16 * (16 * (NT + 3 * NR) + 1) + 16), (size_t)2 * NACC * 256);
}
template <int NT, int NR>
constexpr size_t spatial_reduce_lds() {
  return D8 * (size_t)(NT * NT + 4 * NT * NR) * 256;  // the workgroup reduction
}

// 160 KB of LDS per compute unit, less room for a kernel's static LDS
void allow_lds(const void* fn) {
  (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 159 * 1024);
}

template <int P, int NC>
size_t strip_bytes(size_t frag_values) {
  return D8 * std::max<size_t>(frag_doubles<P>(frag_values) + NW * 16 * strip_ld<NC>(), (size_t)NC * (NC + 1) / 2 * 256);
}

}  // namespace

// the augmentation matrix is the input of the FP64 SVD: FP64 in every mode
void launch_aug_form(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  with_ncb(ncb_of(d.MA), [&](auto c) {
    constexpr int NC = decltype(c)::value;
    constexpr int KS = 4 * NC;
    const size_t lds = strip_bytes<0, NC>(KS * NC * 64);
    hipLaunchKernelGGL((k_aug_form<double, 0, NC, KS>), dim3(d.nwgM, nsd), dim3(NTHR), lds, st, d, axis, sd0);
  });
}

static int dim_cap(const Dev& d, int which) { return which == DIM_M0 ? d.MA : (which == DIM_T ? d.T : d.R); }

void launch_gemm(const Dev& d, int axis, int sd0, int nsd, const void* X, bool x64, int64_t xsd, int rows, int kdim,
                 int ndim, int boff, int bld, void* Y, bool y64, int64_t ysd, const double* rowscale, bool gram,
                 int fill_off, bool rows_are_cells, bool exact, hipStream_t st, bool set_rank, int skip_off) {
  const int nwg = rows_are_cells ? d.nwgN : d.nwgM;
  auto go = [&](auto ti, auto to, auto pc) {
    using SI = typename decltype(ti)::type;
    using SO = typename decltype(to)::type;
    constexpr int P = decltype(pc)::value;
    with_ncb(ncb_of(dim_cap(d, ndim)), [&](auto c) {
      constexpr int NC = decltype(c)::value;
      with_ncb(ncb_of(dim_cap(d, kdim)), [&](auto k) {
        constexpr int KS = sub_cap<P>(decltype(k)::value);
        const size_t lds = strip_bytes<P, NC>(KS * NC * 64);
        hipLaunchKernelGGL((k_gemm<SI, SO, P, NC, KS>), dim3(nwg, nsd), dim3(NTHR), lds, st, d, axis, sd0, X, xsd,
                           rows, kdim, ndim, boff, bld, Y, ysd, rowscale, gram ? 1 : 0, fill_off, set_rank ? 1 : 0, skip_off);
      });
    });
  };
  // FP64 mode: everything FP64.  Mixed modes: the working arrays are FP32;
  // the state and the augmentation matrix stay FP64.
  with_prec(d.prec, exact, [&](auto ts, auto pc) {
    using W = typename decltype(ts)::type;
    if (x64 && y64) go(tag<double>{}, tag<double>{}, pc);
    else if (x64) go(tag<double>{}, tag<W>{}, pc);
    else if (y64) go(tag<W>{}, tag<double>{}, pc);
    else go(tag<W>{}, tag<W>{}, pc);
  });
}

void launch_ang_reduce(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  with_store(d.prec, [&](auto ts) {
    using S = typename decltype(ts)::type;
    with_ncb(ncb_of(d.T), [&](auto ct) {
      constexpr int NT = decltype(ct)::value;
      with_ncb(ncb_of(d.R), [&](auto cr) {
        constexpr int NR = decltype(cr)::value;
        const size_t lds = ang_reduce_lds<NT, NR>();
        if constexpr (NR <= 2 && NT <= 3)  // stored ranks <= 21, intermediate ranks <= 48
          hipLaunchKernelGGL((k_ang_reduce<S, NT, NR>), dim3(d.nwgM, nsd), dim3(NTHR), lds, st, d, axis, sd0);
      });
    });
  });
}

void launch_kstep(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  with_prec(d.prec, false, [&](auto ts, auto pc) {
    using S = typename decltype(ts)::type;
    constexpr int P = decltype(pc)::value;
    with_ksp<P>(d.R, [&](auto kp) {
      constexpr int KSP = decltype(kp)::value;
      with_ncb(ncb_of(d.T), [&](auto c) {
        constexpr int NC = decltype(c)::value;
        const size_t lds = strip_bytes<P, NC>(7 * KSP * NC * 64);
        hipLaunchKernelGGL((k_kstep<S, P, NC, KSP>), dim3(d.nwgN, nsd), dim3(NTHR), lds, st, d, axis, sd0);
      });
    });
  });
}

void launch_spatial_reduce(const Dev& d, int axis, int sd0, int nsd, const void* Q, hipStream_t st) {
  with_store(d.prec, [&](auto ts) {
    using S = typename decltype(ts)::type;
    with_ncb(ncb_of(d.T), [&](auto ct) {
      constexpr int NT = decltype(ct)::value;
      with_ncb(ncb_of(d.R), [&](auto cr) {
        constexpr int NR = decltype(cr)::value;
        const size_t lds = spatial_reduce_lds<NT, NR>();
        if constexpr (NR <= 2 && NT <= 3)  // stored ranks <= 21, intermediate ranks <= 48
          hipLaunchKernelGGL((k_spatial_reduce<S, NT, NR>), dim3(d.nwgN, nsd), dim3(NTHR), lds, st, d, axis, sd0,
                             Q);
      });
    });
  });
}

void launch_lstep(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  with_prec(d.prec, false, [&](auto ts, auto pc) {
    using S = typename decltype(ts)::type;
    constexpr int P = decltype(pc)::value;
    with_ncb(ncb_of(d.T), [&](auto c) {
      constexpr int NC = decltype(c)::value;
      constexpr int KS = sub_cap<P>(NC);
      const size_t lds = strip_bytes<P, NC>(3 * KS * NC * 64);
      hipLaunchKernelGGL((k_lstep<S, P, NC, KS>), dim3(d.nwgM, nsd), dim3(NTHR), lds, st, d, axis, sd0);
    });
  });
}

void launch_coll_kstep(const Dev& d, int sd0, int nsd, hipStream_t st) {
  with_prec(d.prec, false, [&](auto ts, auto pc) {
    using S = typename decltype(ts)::type;
    constexpr int P = decltype(pc)::value;
    // one column beyond the rank carries K.m
    with_ksp<P>(d.R, [&](auto kp) {
      constexpr int KSP = decltype(kp)::value;
      with_ncb(ncb_of(d.R + 1), [&](auto c) {
        constexpr int NC = decltype(c)::value;
        if constexpr (NC <= 2)
          hipLaunchKernelGGL((k_coll_kstep<S, P, NC, KSP>), dim3(d.nwgN, nsd), dim3(NTHR), 0, st, d, sd0);
      });
    });
  });
}

void launch_coll_reduce(const Dev& d, int sd0, int nsd, hipStream_t st) {
  with_ncb(ncb_of(d.R), [&](auto c) {
    constexpr int NC = decltype(c)::value;
    if constexpr (NC <= 2)
      hipLaunchKernelGGL((k_coll_reduce<NC>), dim3(d.nwgN, nsd), dim3(NTHR), 0, st, d, sd0);
  });
}

void launch_coll_lstep(const Dev& d, int sd0, int nsd, hipStream_t st) {
  with_prec(d.prec, false, [&](auto ts, auto pc) {
    using S = typename decltype(ts)::type;
    constexpr int P = decltype(pc)::value;
    if (d.R > CAPR) {
      // the wide plan: stored ranks up to 64
      constexpr int KSP = 16;  // 64 columns: sixteen 4-column steps, or two 32-column BF16 groups
      hipLaunchKernelGGL((k_coll_lstep<S, P, 4, KSP>), dim3(d.nwgM, nsd), dim3(NTHR), 0, st, d, sd0);
      return;
    }
    with_ksp<P>(d.R, [&](auto kp) {
      constexpr int KSP = decltype(kp)::value;
      with_ncb(ncb_of(d.R), [&](auto c) {
        constexpr int NC = decltype(c)::value;
        if constexpr (NC <= 2)
          hipLaunchKernelGGL((k_coll_lstep<S, P, NC, KSP>), dim3(d.nwgM, nsd), dim3(NTHR), 0, st, d, sd0);
      });
    });
  });
}

void launch_moments_twopass(const Dev& d, int nmom, double* smv, double* rho, double* jx, double* jy,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_moments_vec, dim3(d.nsub), dim3(NTHR), 0, st, d, nmom, smv);
  const int nb = (d.N + NTHR - 1) / NTHR;
  hipLaunchKernelGGL(k_moments_apply, dim3(nb < 16 ? nb : 16, d.nsub), dim3(NTHR), 0, st, d, nmom, smv, rho, jx, jy);
}

void launch_moments(const Dev& d, int nmom, hipStream_t st) {
  const int nb = (d.N + NTHR - 1) / NTHR;
  hipLaunchKernelGGL(k_moments, dim3(nb < 16 ? nb : 16, d.nsub), dim3(NTHR), 0, st, d, nmom);
}

// Workgroups per compute unit that stay resident for the heaviest
// tall-skinny kernels of this configuration (the smallest over the K-step,
// its QR products, the spatial reductions and the L-step).
int ts_resident_wgs(const Dev& d) {
  int occ = 1 << 20;
  auto take = [&](const void* fn, size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, NTHR, lds) == hipSuccess && nb > 0)
      occ = std::min(occ, nb);
  };
  with_prec(d.prec, false, [&](auto ts, auto pc) {
    using S = typename decltype(ts)::type;
    constexpr int P = decltype(pc)::value;
    with_ncb(ncb_of(d.T), [&](auto c) {
      constexpr int NC = decltype(c)::value;
      constexpr int KS = 4 * NC;
      with_ksp<P>(d.R, [&](auto kp) {
        constexpr int KSP = decltype(kp)::value;
        take((const void*)k_kstep<S, P, NC, KSP>, strip_bytes<P, NC>(7 * KSP * NC * 64));
      });
      take((const void*)k_lstep<S, P, NC, sub_cap<P>(NC)>, strip_bytes<P, NC>(3 * sub_cap<P>(NC) * NC * 64));
      take((const void*)k_gemm<S, S, 0, NC, KS>, strip_bytes<0, NC>(KS * NC * 64));
      with_ncb(ncb_of(d.R), [&](auto cr) {
        constexpr int NR = decltype(cr)::value;
        if constexpr (NR <= 2 && NC <= 3)
          take((const void*)k_spatial_reduce<S, NC, NR>, spatial_reduce_lds<NC, NR>());
      });
    });
  });
  return occ == (1 << 20) ? 1 : occ;
}

// Allow the dynamically sized kernels the whole LDS of a compute unit.
void init_kernels() {
  for (int prec = 0; prec < 3; ++prec) {
    for (int exact = 0; exact < 2; ++exact) {
      with_prec(prec, exact != 0, [&](auto ts, auto pc) {
        using W = typename decltype(ts)::type;
        constexpr int P = decltype(pc)::value;
        for (int nc = 1; nc <= 4; ++nc) {
          with_ncb(nc, [&](auto c) {
            constexpr int NC = decltype(c)::value;
            allow_lds((const void*)k_aug_form<double, 0, NC, 4 * NC>);
            for (int rc = 1; rc <= CAPR; rc += 4)
              with_ksp<P>(rc, [&](auto kp) { allow_lds((const void*)k_kstep<W, P, NC, decltype(kp)::value>); });
            allow_lds((const void*)k_lstep<W, P, NC, sub_cap<P>(NC)>);
            for (int kc = 1; kc <= 4; ++kc) {
              with_ncb(kc, [&](auto k) {
                constexpr int KS = sub_cap<P>(decltype(k)::value);
                allow_lds((const void*)k_gemm<double, double, P, NC, KS>);
                allow_lds((const void*)k_gemm<double, W, P, NC, KS>);
                allow_lds((const void*)k_gemm<W, double, P, NC, KS>);
                allow_lds((const void*)k_gemm<W, W, P, NC, KS>);
              });
            }
            for (int nr = 1; nr <= 2; ++nr) {
              with_ncb(nr, [&](auto r) {
                constexpr int NR = decltype(r)::value;
                if constexpr (NR <= 2 && NC <= 3) {
                  allow_lds((const void*)k_ang_reduce<W, NC, NR>);
                  allow_lds((const void*)k_spatial_reduce<W, NC, NR>);
                }
              });
            }
          });
        }
      });
    }
  }
  // an attribute the runtime refused would otherwise surface at the first
  // launch check; a kernel that then lacks LDS fails its own launch instead
  (void)hipGetLastError();
}

}  // namespace dd
