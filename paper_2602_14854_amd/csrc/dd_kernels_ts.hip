// Tall-skinny kernels of the DD-DLRA step: every launch covers all
// subdomains of a batch (blockIdx.y) and a strided set of 64-row tiles of the
// cell or direction dimension (blockIdx.x).  Reductions over rows (Gram
// matrices, Galerkin matrices) leave one partial per workgroup; the small
// per-subdomain kernels add the partials in a fixed order, so results are
// bitwise reproducible.
//
// Memory layout (per subdomain, column-major, one column contiguous):
//   cells  p = iy*lnx + ix  -> x-neighbours at p+-1, y-neighbours at p+-lnx
//   directions q            -> rows of V, V-hat, L
// Consecutive threads take consecutive rows, so every global access of a
// column is coalesced for both the x- and the y-stencil.
#include "dd_internal.h"

namespace dd {

constexpr int CAPR = 21;  // largest stored rank (3 * CAPR <= CAP)

// ----------------------------------------------------------------------------
// Augmentation matrix (Algorithm 4, step 1), weighted by sqrt(w) so that the
// plain Gram matrix is L0^T W L0:
//   A[q, :] = sqrt(w_q) [ V[q,:] S^T | V_lo[q,:] S_lo^T | V_hi[q,:] S_hi^T ]
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(NTHR) void k_aug_form(Dev d, int axis, int sd0) {
  const int s = sd0 + blockIdx.y;
  const int nb[3] = {s, neighbour(d, s, axis, -1), neighbour(d, s, axis, +1)};
  int rb[3], cb[3];
  cb[0] = 0;
  for (int b = 0; b < 3; ++b) rb[b] = nb[b] >= 0 ? d.rank[nb[b]] : 0;
  cb[1] = rb[0];
  cb[2] = rb[0] + rb[1];
  const int m0 = rb[0] + rb[1] + rb[2];
  const int M = d.M, R = d.R;

  extern __shared__ double lds[];
  double* Ss = lds;                 // 3 blocks of R x R
  double* Ys = lds + 3 * R * R;     // LDT x MA
  for (int b = 0; b < 3; ++b) {
    if (nb[b] < 0) continue;
    const double* Sb = d.S + (int64_t)nb[b] * R * R;
    for (int idx = threadIdx.x; idx < rb[b] * rb[b]; idx += NTHR) {
      int i = idx % rb[b], k = idx / rb[b];
      Ss[b * R * R + i + k * R] = Sb[i + k * R];
    }
  }
  __syncthreads();

  double* As = d.A + (int64_t)s * M * d.MA;
  GramAcc g;
  g.zero();
  const int i = threadIdx.x % TILE, cg = threadIdx.x / TILE;
  for (int tile = blockIdx.x; tile < d.ntM; tile += gridDim.x) {
    const int q0 = tile * TILE;
    const int nr = min(TILE, M - q0);
    const int q = q0 + i;
    for (int j = cg; j < m0; j += NTHR / TILE) {
      const int b = (j >= cb[2]) ? 2 : ((j >= cb[1]) ? 1 : 0);
      const int jl = j - cb[b];
      double acc = 0.0;
      if (i < nr) {
        const double* Vb = d.V + (int64_t)nb[b] * M * R;
        const double* Sb = Ss + b * R * R;
        for (int k = 0; k < rb[b]; ++k) acc = fma(Vb[(int64_t)k * M + q], Sb[jl + k * R], acc);
        acc *= d.sw[q];
        As[(int64_t)j * M + q] = acc;
      }
      Ys[i + j * LDT] = (i < nr) ? acc : 0.0;
    }
    __syncthreads();
    g.add(Ys, LDT, nr, m0);
    __syncthreads();
  }
  g.store(gpart_of(d, s) + (int64_t)blockIdx.x * d.gpTile, m0);
}

void launch_aug_form(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  const size_t lds = sizeof(double) * (3 * d.R * d.R + LDT * d.MA);
  hipLaunchKernelGGL(k_aug_form, dim3(d.nwgM, nsd), dim3(NTHR), lds, st, d, axis, sd0);
}

// ----------------------------------------------------------------------------
// Generic tall-skinny product Y = diag(rowscale) X B with an optional
// partial Gram matrix of Y.  X is rows x k, B is k x n (small workspace,
// leading dimension bld).  Columns flagged in the fill mask are replaced by
// deterministic pseudo-random values (used to complete a basis where the
// augmentation matrix has no information).
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(NTHR) void k_gemm(Dev d, int axis, int sd0, const double* X, int64_t xsd,
                                               int rows, int kdim, int ndim, int boff, int bld,
                                               double* Y, int64_t ysd, const double* rowscale, int gram,
                                               int fill_off, int ntiles, int kc) {
  const int s = sd0 + blockIdx.y;
  const int k = dim_of(d, s, axis, kdim);
  const int n = dim_of(d, s, axis, ndim);
  extern __shared__ double lds[];
  double* Bs = lds;                   // kc x n (leading dimension kc)
  double* Xs = lds + kc * CAP;        // LDT x max(kc, n)
  __shared__ int fillm[CAP];
  const double* sm = small_of(d, s);
  for (int idx = threadIdx.x; idx < k * n; idx += NTHR) {
    int c = idx % k, j = idx / k;
    Bs[c + j * kc] = sm[boff + c + j * bld];
  }
  for (int j = threadIdx.x; j < CAP; j += NTHR) fillm[j] = (fill_off >= 0 && j < n) ? (sm[fill_off + j] != 0.0) : 0;
  __syncthreads();

  const double* Xsd = X + (int64_t)s * xsd;
  double* Ysd = Y + (int64_t)s * ysd;
  GramAcc g;
  g.zero();
  const int i = threadIdx.x % TILE, cg = threadIdx.x / TILE;
  constexpr int NJ = CAP / (NTHR / TILE);
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int r0 = tile * TILE;
    const int nr = min(TILE, rows - r0);
    for (int idx = threadIdx.x; idx < TILE * k; idx += NTHR) {
      int ii = idx % TILE, c = idx / TILE;
      Xs[ii + c * LDT] = (ii < nr) ? Xsd[(int64_t)c * rows + r0 + ii] : 0.0;
    }
    __syncthreads();
    double acc[NJ];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) acc[jj] = 0.0;
    for (int c = 0; c < k; ++c) {
      const double x = Xs[i + c * LDT];
#pragma unroll
      for (int jj = 0; jj < NJ; ++jj) {
        const int j = cg + jj * (NTHR / TILE);
        if (j < n) acc[jj] = fma(x, Bs[c + j * kc], acc[jj]);
      }
    }
    __syncthreads();
    const int row = r0 + i;
    const double rs = (rowscale != nullptr && i < nr) ? rowscale[row] : 1.0;
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      const int j = cg + jj * (NTHR / TILE);
      if (j < n) {
        double v = acc[jj] * rs;
        if (fillm[j]) v = hash_unit(((uint64_t)s << 40) ^ ((uint64_t)j << 24) ^ (uint64_t)row);
        if (i < nr) Ysd[(int64_t)j * rows + row] = v;
        Xs[i + j * LDT] = (i < nr) ? v : 0.0;
      }
    }
    __syncthreads();
    if (gram) g.add(Xs, LDT, nr, n);
    __syncthreads();
  }
  if (gram) g.store(gpart_of(d, s) + (int64_t)blockIdx.x * d.gpTile, n);
}

void launch_gemm(const Dev& d, int axis, int sd0, int nsd, const double* X, int64_t xsd, int rows,
                 int kdim, int ndim, int boff, int bld, double* Y, int64_t ysd, const double* rowscale,
                 bool gram, int fill_off, bool rows_are_cells, hipStream_t st) {
  const int nwg = rows_are_cells ? d.nwgN : d.nwgM;
  const int nt = rows_are_cells ? d.ntN : d.ntM;
  auto cap = [&](int which) { return which == DIM_M0 ? d.MA : (which == DIM_T ? d.T : d.R); };
  const int kc = cap(kdim), nc = cap(ndim);
  const size_t lds = sizeof(double) * ((size_t)kc * CAP + (size_t)LDT * (kc > nc ? kc : nc));
  hipLaunchKernelGGL(k_gemm, dim3(nwg, nsd), dim3(NTHR), lds, st, d, axis, sd0, X, xsd, rows, kdim, ndim,
                     boff, bld, Y, ysd, rowscale, gram ? 1 : 0, fill_off, nt, kc);
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
__global__ __launch_bounds__(NTHR) void k_ang_reduce(Dev d, int axis, int sd0) {
  const int s = sd0 + blockIdx.y;
  const int lo = neighbour(d, s, axis, -1), hi = neighbour(d, s, axis, +1);
  const int r = d.rank[s], rl = lo >= 0 ? d.rank[lo] : 0, rh = hi >= 0 ? d.rank[hi] : 0;
  const int t = d.tdim[s];
  const int M = d.M, R = d.R, T = d.T;
  const double* om = axis == 0 ? d.omx : d.omy;
  extern __shared__ double lds[];
  double* Qs = lds;                       // LDT x T
  double* Vs = lds + LDT * T;             // LDT x 3R
  double* oms = Vs + LDT * 3 * R;         // TILE

  double* out = gpart_of(d, s) + (int64_t)blockIdx.x * d.gpTile;
  const int oT = 0, oC = R * T, oEp = oC + T * T, oEn = oEp + T * T, oOlo = oEn + T * T, oOhi = oOlo + R * T;
  const int nT = r * t, nC = t * t, nOl = rl * t, nOh = rh * t;
  const int ntot = nT + 3 * nC + nOl + nOh;
  for (int e = threadIdx.x; e < ntot; e += NTHR) {
    int o;
    if (e < nT) o = oT + (e % r) + (e / r) * R;
    else if (e < nT + nC) { int ee = e - nT; o = oC + ee; }
    else if (e < nT + 2 * nC) { int ee = e - nT - nC; o = oEp + ee; }
    else if (e < nT + 3 * nC) { int ee = e - nT - 2 * nC; o = oEn + ee; }
    else if (e < nT + 3 * nC + nOl) { int ee = e - nT - 3 * nC; o = oOlo + (ee % rl) + (ee / rl) * R; }
    else { int ee = e - nT - 3 * nC - nOl; o = oOhi + (ee % rh) + (ee / rh) * R; }
    out[o] = 0.0;
  }
  const double* Qsd = d.Qh + (int64_t)s * M * T;
  const double* Vo = d.V + (int64_t)s * M * R;
  const double* Vl = lo >= 0 ? d.V + (int64_t)lo * M * R : nullptr;
  const double* Vh = hi >= 0 ? d.V + (int64_t)hi * M * R : nullptr;
  for (int tile = blockIdx.x; tile < d.ntM; tile += gridDim.x) {
    const int q0 = tile * TILE;
    const int nr = min(TILE, M - q0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < TILE * t; idx += NTHR) {
      int ii = idx % TILE, c = idx / TILE;
      Qs[ii + c * LDT] = ii < nr ? Qsd[(int64_t)c * M + q0 + ii] : 0.0;
    }
    const int rv = r + rl + rh;
    for (int idx = threadIdx.x; idx < TILE * rv; idx += NTHR) {
      int ii = idx % TILE, c = idx / TILE;
      double v = 0.0;
      if (ii < nr) {
        const int q = q0 + ii;
        if (c < r) v = Vo[(int64_t)c * M + q];
        else if (c < r + rl) v = Vl[(int64_t)(c - r) * M + q];
        else v = Vh[(int64_t)(c - r - rl) * M + q];
        v *= d.sw[q];
      }
      Vs[ii + c * LDT] = v;
    }
    for (int ii = threadIdx.x; ii < TILE; ii += NTHR) {
      oms[ii] = ii < nr ? om[q0 + ii] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ntot; e += NTHR) {
      double acc = 0.0;
      int o;
      if (e < nT) {
        const int a = e % r, b = e / r;
        for (int q = 0; q < nr; ++q) acc = fma(Vs[q + a * LDT], Qs[q + b * LDT], acc);
        o = oT + a + b * R;
      } else if (e < nT + 3 * nC) {
        const int blk = (e - nT) / nC, ee = (e - nT) % nC;
        const int a = ee % t, b = ee / t;
        if (blk == 0) {
          for (int q = 0; q < nr; ++q) acc = fma(Qs[q + a * LDT] * oms[q], Qs[q + b * LDT], acc);
          o = oC + a + b * t;
        } else if (blk == 1) {
          for (int q = 0; q < nr; ++q)
            if (oms[q] >= 0.0) acc = fma(Qs[q + a * LDT], Qs[q + b * LDT], acc);
          o = oEp + a + b * t;
        } else {
          for (int q = 0; q < nr; ++q)
            if (oms[q] < 0.0) acc = fma(Qs[q + a * LDT], Qs[q + b * LDT], acc);
          o = oEn + a + b * t;
        }
      } else if (e < nT + 3 * nC + nOl) {
        const int ee = e - nT - 3 * nC;
        const int a = ee % rl, b = ee / rl;
        for (int q = 0; q < nr; ++q)
          if (oms[q] >= 0.0 && q < nr) acc = fma(Vs[q + (r + a) * LDT], Qs[q + b * LDT], acc);
        o = oOlo + a + b * R;
      } else {
        const int ee = e - nT - 3 * nC - nOl;
        const int a = ee % rh, b = ee / rh;
        for (int q = 0; q < nr; ++q)
          if (oms[q] < 0.0) acc = fma(Vs[q + (r + rl + a) * LDT], Qs[q + b * LDT], acc);
        o = oOhi + a + b * R;
      }
      out[o] += acc;
    }
  }
}

void launch_ang_reduce(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  const size_t lds = sizeof(double) * ((size_t)LDT * (d.T + 3 * d.R) + TILE);
  hipLaunchKernelGGL(k_ang_reduce, dim3(d.nwgM, nsd), dim3(NTHR), lds, st, d, axis, sd0);
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
__global__ __launch_bounds__(NTHR) void k_kstep(Dev d, int axis, int sd0) {
  const int s = sd0 + blockIdx.y;
  const int lo = neighbour(d, s, axis, -1), hi = neighbour(d, s, axis, +1);
  const int r = d.rank[s], rl = lo >= 0 ? d.rank[lo] : 0, rh = hi >= 0 ? d.rank[hi] : 0;
  const int t = d.tdim[s];
  const int N = d.N, R = d.R;
  const int T = d.T;
  extern __shared__ double lds[];
  double* Cf = lds;                 // 7 blocks of R x T (leading dimension R)
  double* Ks = lds + 7 * R * T;     // LDT x T
  const double* sm = small_of(d, s);
  const int offs[7] = {d.oM0, d.oMm, d.oMp, d.oGLo, d.oGHi, d.oGLoN, d.oGHiN};
  const int rows[7] = {r, r, r, r, r, rl, rh};
  for (int m = 0; m < 7; ++m) {
    for (int idx = threadIdx.x; idx < rows[m] * t; idx += NTHR) {
      int c = idx % rows[m], j = idx / rows[m];
      Cf[m * R * T + c + j * R] = sm[offs[m] + c + j * R];
    }
  }
  __syncthreads();
  const double* M0 = Cf;
  const double* Mm = Cf + 1 * R * T;
  const double* Mp = Cf + 2 * R * T;
  const double* GLo = Cf + 3 * R * T;
  const double* GHi = Cf + 4 * R * T;
  const double* GLoN = Cf + 5 * R * T;
  const double* GHiN = Cf + 6 * R * T;

  const double* Us = d.U + (int64_t)s * N * R;
  const double* Ul = lo >= 0 ? d.U + (int64_t)lo * N * R : nullptr;
  const double* Uh = hi >= 0 ? d.U + (int64_t)hi * N * R : nullptr;
  double* K1 = d.K1 + (int64_t)s * N * T;
  const int e = axis == 0 ? 1 : d.lnx;
  const int na = axis == 0 ? d.lnx : d.lny;
  GramAcc g;
  g.zero();
  const int i = threadIdx.x % TILE, cg = threadIdx.x / TILE;
  constexpr int NJ = CAP / (NTHR / TILE);
  for (int tile = blockIdx.x; tile < d.ntN; tile += gridDim.x) {
    const int p0 = tile * TILE;
    const int nr = min(TILE, N - p0);
    const int p = p0 + i;
    double acc[NJ];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) acc[jj] = 0.0;
    if (i < nr) {
      const int ix = p % d.lnx, iy = p / d.lnx;
      const int ia = axis == 0 ? ix : iy;
      const int f = axis == 0 ? iy : ix;
      for (int c = 0; c < r; ++c) {
        const double u = Us[(int64_t)c * N + p];
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
          const int j = cg + jj * (NTHR / TILE);
          if (j < t) acc[jj] = fma(u, M0[c + j * R], acc[jj]);
        }
      }
      if (ia > 0) {
        for (int c = 0; c < r; ++c) {
          const double u = Us[(int64_t)c * N + p - e];
#pragma unroll
          for (int jj = 0; jj < NJ; ++jj) {
            const int j = cg + jj * (NTHR / TILE);
            if (j < t) acc[jj] = fma(u, Mm[c + j * R], acc[jj]);
          }
        }
      } else {
        for (int c = 0; c < r; ++c) {
          const double u = Us[(int64_t)c * N + p];
#pragma unroll
          for (int jj = 0; jj < NJ; ++jj) {
            const int j = cg + jj * (NTHR / TILE);
            if (j < t) acc[jj] = fma(u, GLo[c + j * R], acc[jj]);
          }
        }
        if (lo >= 0) {
          const int pn = face_cell(d, axis, true, f);
          for (int c = 0; c < rl; ++c) {
            const double u = Ul[(int64_t)c * N + pn];
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj) {
              const int j = cg + jj * (NTHR / TILE);
              if (j < t) acc[jj] = fma(u, GLoN[c + j * R], acc[jj]);
            }
          }
        }
      }
      if (ia < na - 1) {
        for (int c = 0; c < r; ++c) {
          const double u = Us[(int64_t)c * N + p + e];
#pragma unroll
          for (int jj = 0; jj < NJ; ++jj) {
            const int j = cg + jj * (NTHR / TILE);
            if (j < t) acc[jj] = fma(u, Mp[c + j * R], acc[jj]);
          }
        }
      } else {
        for (int c = 0; c < r; ++c) {
          const double u = Us[(int64_t)c * N + p];
#pragma unroll
          for (int jj = 0; jj < NJ; ++jj) {
            const int j = cg + jj * (NTHR / TILE);
            if (j < t) acc[jj] = fma(u, GHi[c + j * R], acc[jj]);
          }
        }
        if (hi >= 0) {
          const int pn = face_cell(d, axis, false, f);
          for (int c = 0; c < rh; ++c) {
            const double u = Uh[(int64_t)c * N + pn];
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj) {
              const int j = cg + jj * (NTHR / TILE);
              if (j < t) acc[jj] = fma(u, GHiN[c + j * R], acc[jj]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      const int j = cg + jj * (NTHR / TILE);
      if (j < t) {
        if (i < nr) K1[(int64_t)j * N + p] = acc[jj];
        Ks[i + j * LDT] = (i < nr) ? acc[jj] : 0.0;
      }
    }
    __syncthreads();
    g.add(Ks, LDT, nr, t);
    __syncthreads();
  }
  g.store(gpart_of(d, s) + (int64_t)blockIdx.x * d.gpTile, t);
}

void launch_kstep(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  const size_t lds = sizeof(double) * ((size_t)7 * d.R * d.T + (size_t)LDT * d.T);
  hipLaunchKernelGGL(k_kstep, dim3(d.nwgN, nsd), dim3(NTHR), lds, st, d, axis, sd0);
}

// ----------------------------------------------------------------------------
// Spatial Galerkin matrices of the S- and L-steps (eqs. advx_evolS/L):
//   Gm[i,j] = sum_p Q[p,i] (Q[p,j] - Q[p-e,j])   (zero beyond the low face)
//   Gp[i,j] = sum_p Q[p,i] (Q[p+e,j] - Q[p,j])   (zero beyond the high face)
// with Q = h U^1; dividing by h gives h^2 U^T D-+_0 U.  Partial layout:
// Gm @0, Gp @T*T, both t x t with leading dimension t.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(NTHR) void k_spatial_reduce(Dev d, int axis, int sd0, const double* Q) {
  const int s = sd0 + blockIdx.y;
  const int t = d.tdim[s];
  const int N = d.N, T = d.T;
  extern __shared__ double lds[];
  double* Qs = lds;                 // LDT x T each
  double* Dm = lds + LDT * T;
  double* Dp = lds + 2 * LDT * T;
  const double* Qsd = Q + (int64_t)s * N * T;
  double* out = gpart_of(d, s) + (int64_t)blockIdx.x * d.gpTile;
  for (int e2 = threadIdx.x; e2 < 2 * t * t; e2 += NTHR) out[(e2 < t * t) ? e2 : (T * T + e2 - t * t)] = 0.0;
  const int e = axis == 0 ? 1 : d.lnx;
  const int na = axis == 0 ? d.lnx : d.lny;
  for (int tile = blockIdx.x; tile < d.ntN; tile += gridDim.x) {
    const int p0 = tile * TILE;
    const int nr = min(TILE, N - p0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < TILE * t; idx += NTHR) {
      const int ii = idx % TILE, c = idx / TILE;
      double q = 0.0, qm = 0.0, qp = 0.0;
      if (ii < nr) {
        const int p = p0 + ii;
        const int ia = axis == 0 ? (p % d.lnx) : (p / d.lnx);
        q = Qsd[(int64_t)c * N + p];
        qm = q - (ia > 0 ? Qsd[(int64_t)c * N + p - e] : 0.0);
        qp = (ia < na - 1 ? Qsd[(int64_t)c * N + p + e] : 0.0) - q;
      }
      Qs[ii + c * LDT] = q;
      Dm[ii + c * LDT] = qm;
      Dp[ii + c * LDT] = qp;
    }
    __syncthreads();
    for (int e2 = threadIdx.x; e2 < 2 * t * t; e2 += NTHR) {
      const int blk = e2 / (t * t), ee = e2 % (t * t);
      const int a = ee % t, b = ee / t;
      const double* D = blk == 0 ? Dm : Dp;
      double acc = 0.0;
      for (int q = 0; q < nr; ++q) acc = fma(Qs[q + a * LDT], D[q + b * LDT], acc);
      out[blk * T * T + ee] += acc;
    }
  }
}

void launch_spatial_reduce(const Dev& d, int axis, int sd0, int nsd, const double* Q, hipStream_t st) {
  const size_t lds = sizeof(double) * 3 * (size_t)LDT * d.T;
  hipLaunchKernelGGL(k_spatial_reduce, dim3(d.nwgN, nsd), dim3(NTHR), lds, st, d, axis, sd0, Q);
}

// ----------------------------------------------------------------------------
// L-step of an advection stage (eq. advx_evolL), weighted by sqrt(w):
//   AL[q,:] = Qh[q,:] (P0 + Omega_q^+ Pm + Omega_q^- Pp)
// with P0 = S2^T, Pm = -dt c Hm^T, Pp = -dt c Hp^T; each direction is
// upwinded by the sign of its own Omega.  Leaves the partial Gram of AL.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(NTHR) void k_lstep(Dev d, int axis, int sd0) {
  const int s = sd0 + blockIdx.y;
  const int t = d.tdim[s];
  const int M = d.M, T = d.T;
  const double* om = axis == 0 ? d.omx : d.omy;
  extern __shared__ double lds[];
  double* P = lds;                  // 3 blocks of T x T (leading dimension T)
  double* Xs = lds + 3 * T * T;     // LDT x T
  const double* sm = small_of(d, s);
  for (int idx = threadIdx.x; idx < t * t; idx += NTHR) {
    const int c = idx % t, j = idx / t;
    P[c + j * T] = sm[d.oP0 + c + j * T];
    P[T * T + c + j * T] = sm[d.oPm + c + j * T];
    P[2 * T * T + c + j * T] = sm[d.oPp + c + j * T];
  }
  __syncthreads();
  const double* Qsd = d.Qh + (int64_t)s * M * T;
  double* ALs = d.AL + (int64_t)s * M * T;
  GramAcc g;
  g.zero();
  const int i = threadIdx.x % TILE, cg = threadIdx.x / TILE;
  constexpr int NJ = CAP / (NTHR / TILE);
  for (int tile = blockIdx.x; tile < d.ntM; tile += gridDim.x) {
    const int q0 = tile * TILE;
    const int nr = min(TILE, M - q0);
    for (int idx = threadIdx.x; idx < TILE * t; idx += NTHR) {
      const int ii = idx % TILE, c = idx / TILE;
      Xs[ii + c * LDT] = ii < nr ? Qsd[(int64_t)c * M + q0 + ii] : 0.0;
    }
    __syncthreads();
    const int q = q0 + i;
    const double o = (i < nr) ? om[q] : 0.0;
    const double* Ps = (o >= 0.0) ? P + T * T : P + 2 * T * T;
    double acc[NJ];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) acc[jj] = 0.0;
    for (int c = 0; c < t; ++c) {
      const double x = Xs[i + c * LDT];
#pragma unroll
      for (int jj = 0; jj < NJ; ++jj) {
        const int j = cg + jj * (NTHR / TILE);
        if (j < t) acc[jj] = fma(x, fma(o, Ps[c + j * T], P[c + j * T]), acc[jj]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      const int j = cg + jj * (NTHR / TILE);
      if (j < t) {
        if (i < nr) ALs[(int64_t)j * M + q] = acc[jj];
        Xs[i + j * LDT] = (i < nr) ? acc[jj] : 0.0;
      }
    }
    __syncthreads();
    g.add(Xs, LDT, nr, t);
    __syncthreads();
  }
  g.store(gpart_of(d, s) + (int64_t)blockIdx.x * d.gpTile, t);
}

void launch_lstep(const Dev& d, int axis, int sd0, int nsd, hipStream_t st) {
  const size_t lds = sizeof(double) * ((size_t)3 * d.T * d.T + (size_t)LDT * d.T);
  hipLaunchKernelGGL(k_lstep, dim3(d.nwgM, nsd), dim3(NTHR), lds, st, d, axis, sd0);
}

// ----------------------------------------------------------------------------
// Collision stage K-step (eq. coll_evolK), K = U S, m = V^T w:
//   K1[p] = (1 - dt c_t[p]) K[p] + dt (c_s[p]/W) (K[p].m) m + dt Q[p] m
// Leaves the partial Gram of K1 (r columns).
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(NTHR) void k_coll_kstep(Dev d, int sd0) {
  const int s = sd0 + blockIdx.y;
  const int r = d.rank[s];
  const int N = d.N, R = d.R;
  __shared__ double Ss[CAPR * CAPR];
  __shared__ double mv[CAPR];
  __shared__ double Ks[LDT * CAPR];
  const double* sm = small_of(d, s);
  const double* Sg = d.S + (int64_t)s * R * R;
  for (int idx = threadIdx.x; idx < r * r; idx += NTHR) {
    const int a = idx % r, b = idx / r;
    Ss[a + b * CAPR] = Sg[a + b * R];
  }
  for (int a = threadIdx.x; a < r; a += NTHR) mv[a] = sm[d.oMv + a];
  __syncthreads();
  const double* Us = d.U + (int64_t)s * N * R;
  const double* cs = d.cs + (int64_t)s * N;
  const double* ct = d.ct + (int64_t)s * N;
  const double* Qs = d.Qsrc + (int64_t)s * N;
  double* K1 = d.K1 + (int64_t)s * N * d.T;
  const double dt = d.dt, iW = 1.0 / d.W;
  GramAcc g;
  g.zero();
  const int i = threadIdx.x % TILE, cg = threadIdx.x / TILE;
  for (int tile = blockIdx.x; tile < d.ntN; tile += gridDim.x) {
    const int p0 = tile * TILE;
    const int nr = min(TILE, N - p0);
    const int p = p0 + i;
    double Kp[CAPR];
#pragma unroll
    for (int b = 0; b < CAPR; ++b) Kp[b] = 0.0;
    double km = 0.0;
    if (i < nr) {
      for (int a = 0; a < r; ++a) {
        const double u = Us[(int64_t)a * N + p];
#pragma unroll
        for (int b = 0; b < CAPR; ++b)
          if (b < r) Kp[b] = fma(u, Ss[a + b * CAPR], Kp[b]);
      }
#pragma unroll
      for (int b = 0; b < CAPR; ++b)
        if (b < r) km = fma(Kp[b], mv[b], km);
    }
    const double a0 = (i < nr) ? 1.0 - dt * ct[p] : 0.0;
    const double a1 = (i < nr) ? dt * (cs[p] * iW * km + Qs[p]) : 0.0;
#pragma unroll
    for (int b = 0; b < CAPR; ++b) {
      if (b < r && (b % (NTHR / TILE)) == cg) {
        const double v = (i < nr) ? fma(a0, Kp[b], a1 * mv[b]) : 0.0;
        if (i < nr) K1[(int64_t)b * N + p] = v;
        Ks[i + b * LDT] = v;
      }
    }
    __syncthreads();
    g.add(Ks, LDT, nr, r);
    __syncthreads();
  }
  g.store(gpart_of(d, s) + (int64_t)blockIdx.x * d.gpTile, r);
}

void launch_coll_kstep(const Dev& d, int sd0, int nsd, hipStream_t st) {
  hipLaunchKernelGGL(k_coll_kstep, dim3(d.nwgN, nsd), dim3(NTHR), 0, st, d, sd0);
}

// ----------------------------------------------------------------------------
// Collision Galerkin reductions (eq. coll_evolS/L) from U^1 (already in the
// state buffer):  Gs = h^2 U^T diag(c_s) U,  Gt = h^2 U^T diag(c_t) U,
// qv = h^2 U^T Q.  Partial layout: Gs @0, Gt @R*R (ld R), qv @2R*R.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(NTHR) void k_coll_reduce(Dev d, int sd0) {
  const int s = sd0 + blockIdx.y;
  const int r = d.rank[s];
  const int N = d.N, R = d.R;
  __shared__ double Us[LDT * CAPR];
  __shared__ double w3[3 * TILE];
  const double* Ug = d.U + (int64_t)s * N * R;
  const double* cs = d.cs + (int64_t)s * N;
  const double* ct = d.ct + (int64_t)s * N;
  const double* Qg = d.Qsrc + (int64_t)s * N;
  double* out = gpart_of(d, s) + (int64_t)blockIdx.x * d.gpTile;
  const int ntot = 2 * r * r + r;
  for (int e = threadIdx.x; e < ntot; e += NTHR) {
    int o;
    if (e < 2 * r * r) { const int blk = e / (r * r), ee = e % (r * r); o = blk * R * R + (ee % r) + (ee / r) * R; }
    else o = 2 * R * R + (e - 2 * r * r);
    out[o] = 0.0;
  }
  const double h2 = d.h * d.h;
  for (int tile = blockIdx.x; tile < d.ntN; tile += gridDim.x) {
    const int p0 = tile * TILE;
    const int nr = min(TILE, N - p0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < TILE * r; idx += NTHR) {
      const int ii = idx % TILE, c = idx / TILE;
      Us[ii + c * LDT] = ii < nr ? Ug[(int64_t)c * N + p0 + ii] : 0.0;
    }
    for (int ii = threadIdx.x; ii < TILE; ii += NTHR) {
      w3[ii] = ii < nr ? cs[p0 + ii] : 0.0;
      w3[TILE + ii] = ii < nr ? ct[p0 + ii] : 0.0;
      w3[2 * TILE + ii] = ii < nr ? Qg[p0 + ii] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ntot; e += NTHR) {
      double acc = 0.0;
      int o;
      if (e < 2 * r * r) {
        const int blk = e / (r * r), ee = e % (r * r);
        const int a = ee % r, b = ee / r;
        const double* wt = w3 + blk * TILE;
        for (int q = 0; q < nr; ++q) acc = fma(Us[q + a * LDT] * wt[q], Us[q + b * LDT], acc);
        o = blk * R * R + a + b * R;
      } else {
        const int a = e - 2 * r * r;
        for (int q = 0; q < nr; ++q) acc = fma(Us[q + a * LDT], w3[2 * TILE + q], acc);
        o = 2 * R * R + a;
      }
      out[o] += h2 * acc;
    }
  }
}

void launch_coll_reduce(const Dev& d, int sd0, int nsd, hipStream_t st) {
  hipLaunchKernelGGL(k_coll_reduce, dim3(d.nwgN, nsd), dim3(NTHR), 0, st, d, sd0);
}

// ----------------------------------------------------------------------------
// Collision L-step (eq. coll_evolL), weighted by sqrt(w):
//   AL[q,:] = sqrt(w_q) (V[q,:] P + crow),  P = S2^T (I - dt Gt),
//   crow = dt ((S2 m)^T Gs / W + q^T).  Leaves the partial Gram of AL.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(NTHR) void k_coll_lstep(Dev d, int sd0) {
  const int s = sd0 + blockIdx.y;
  const int r = d.rank[s];
  const int M = d.M, R = d.R;
  __shared__ double Ps[CAPR * CAPR];
  __shared__ double cr[CAPR];
  __shared__ double Xs[LDT * CAPR];
  const double* sm = small_of(d, s);
  for (int idx = threadIdx.x; idx < r * r; idx += NTHR) {
    const int a = idx % r, b = idx / r;
    Ps[a + b * CAPR] = sm[d.oP0 + a + b * R];
  }
  for (int a = threadIdx.x; a < r; a += NTHR) cr[a] = sm[d.oCrow + a];
  __syncthreads();
  const double* Vs = d.V + (int64_t)s * M * R;
  double* ALs = d.AL + (int64_t)s * M * d.T;
  GramAcc g;
  g.zero();
  const int i = threadIdx.x % TILE, cg = threadIdx.x / TILE;
  for (int tile = blockIdx.x; tile < d.ntM; tile += gridDim.x) {
    const int q0 = tile * TILE;
    const int nr = min(TILE, M - q0);
    for (int idx = threadIdx.x; idx < TILE * r; idx += NTHR) {
      const int ii = idx % TILE, c = idx / TILE;
      Xs[ii + c * LDT] = ii < nr ? Vs[(int64_t)c * M + q0 + ii] : 0.0;
    }
    __syncthreads();
    const int q = q0 + i;
    double acc[CAPR];
#pragma unroll
    for (int b = 0; b < CAPR; ++b) acc[b] = 0.0;
    for (int c = 0; c < r; ++c) {
      const double x = Xs[i + c * LDT];
#pragma unroll
      for (int b = 0; b < CAPR; ++b)
        if (b < r) acc[b] = fma(x, Ps[c + b * CAPR], acc[b]);
    }
    const double swq = (i < nr) ? d.sw[q] : 0.0;
    __syncthreads();
#pragma unroll
    for (int b = 0; b < CAPR; ++b) {
      if (b < r && (b % (NTHR / TILE)) == cg) {
        const double v = swq * (acc[b] + cr[b]);
        if (i < nr) ALs[(int64_t)b * M + q] = v;
        Xs[i + b * LDT] = (i < nr) ? v : 0.0;
      }
    }
    __syncthreads();
    g.add(Xs, LDT, nr, r);
    __syncthreads();
  }
  g.store(gpart_of(d, s) + (int64_t)blockIdx.x * d.gpTile, r);
}

void launch_coll_lstep(const Dev& d, int sd0, int nsd, hipStream_t st) {
  hipLaunchKernelGGL(k_coll_lstep, dim3(d.nwgM, nsd), dim3(NTHR), 0, st, d, sd0);
}

// ----------------------------------------------------------------------------
// Scalar flux rho = U (S (V^T w)) on the global grid (Section 2).
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(NTHR) void k_moments(Dev d) {
  const int s = blockIdx.y;
  const int r = d.rank[s];
  const int N = d.N, M = d.M, R = d.R;
  __shared__ double mv[CAPR];
  __shared__ double smv[CAPR];
  __shared__ double red[NTHR];
  const double* Vs = d.V + (int64_t)s * M * R;
  for (int a = 0; a < r; ++a) {
    double acc = 0.0;
    for (int q = threadIdx.x; q < M; q += NTHR) acc = fma(Vs[(int64_t)a * M + q], d.w[q], acc);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = NTHR / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) mv[a] = red[0];
    __syncthreads();
  }
  const double* Sg = d.S + (int64_t)s * R * R;
  for (int a = threadIdx.x; a < r; a += NTHR) {
    double acc = 0.0;
    for (int b = 0; b < r; ++b) acc = fma(Sg[a + b * R], mv[b], acc);
    smv[a] = acc;
  }
  __syncthreads();
  const double* Us = d.U + (int64_t)s * N * R;
  const int sx = s % d.px, sy = s / d.px;
  for (int p = blockIdx.x * NTHR + threadIdx.x; p < N; p += gridDim.x * NTHR) {
    double acc = 0.0;
    for (int a = 0; a < r; ++a) acc = fma(Us[(int64_t)a * N + p], smv[a], acc);
    const int ix = p % d.lnx, iy = p / d.lnx;
    d.rho[(int64_t)(sy * d.lny + iy) * d.nx + sx * d.lnx + ix] = acc;
  }
}

void launch_moments(const Dev& d, hipStream_t st) {
  const int nb = (d.N + NTHR - 1) / NTHR;
  hipLaunchKernelGGL(k_moments, dim3(nb < 16 ? nb : 16, d.nsub), dim3(NTHR), 0, st, d);
}

// Allow the dynamically sized kernels the whole LDS of a compute unit.
void init_kernels() {
  const int max_lds = 160 * 1024;
  (void)hipFuncSetAttribute((const void*)k_aug_form, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
  (void)hipFuncSetAttribute((const void*)k_gemm, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds - 256);
  (void)hipFuncSetAttribute((const void*)k_ang_reduce, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
  (void)hipFuncSetAttribute((const void*)k_kstep, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
  (void)hipFuncSetAttribute((const void*)k_spatial_reduce, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
  (void)hipFuncSetAttribute((const void*)k_lstep, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
}

}  // namespace dd
