// Internal definitions shared by the HIP translation units of the DD-DLRA
// engine.  Nothing here is part of the public C ABI (include/dd_dlra.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dd {

constexpr int NTHR = 256;        // threads per workgroup (4 wavefronts of 64)
constexpr int TILE = 64;         // rows per workgroup pass of the tall-skinny kernels
constexpr int CAP = 64;          // largest T (intermediate rank) and MA (= r + r_lo + r_hi)

// error bits latched in Dev::flags
enum : unsigned {
  FLAG_NONFINITE = 1u,
  FLAG_JACOBI_NOCONV = 4u,
  FLAG_RANK_CLAMP = 8u,
};

// which per-subdomain dimension a generic kernel uses
enum Dim : int { DIM_M0 = 0, DIM_T = 1, DIM_R = 2, DIM_RNEW = 3 };

// Everything a kernel needs, passed by value.  Pointers are device memory.
struct Dev {
  // geometry and physics
  int px, py, lnx, lny, N, M, nsub;
  double h, dt, c, W;
  // capacities and launch shapes
  int R, T, MA;
  int ntN, ntM;            // tiles over cells / over directions
  int nwgN, nwgM;          // workgroups per subdomain for cell / direction kernels
  int xpN, xpM;            // partial sums (row splits) of the wide plan's reductions read by wide kernels
  int xgN, xgM;            // the same for the Galerkin job sets and the Gram of A (at most 8)
  int gpTile;              // doubles per workgroup partial
  int64_t gpStride;        // doubles of partials per subdomain (room for the largest grid)
  int64_t smallStride;     // doubles of small workspace per subdomain
  // rank rules and precision mode (DD_PREC_*)
  int rank_mode, r_fixed, r_min, r_max, r_int_max, strict;
  int prec;
  int wide;                // 1: the wide launch plan (capacities beyond the narrow kernels)
  int rk4;                 // 1: every substep is one classic RK4 step (wide plan, FP64)
  int bc_in[4];            // faces -x, +x, -y, +y with a prescribed inflow
  int npseudo;             // their layer slots after the subdomains in U, V, S, rank
  int face;                // cells on the longer subdomain face (ghost rows)
  double tol, tol_aug_rel;
  // state (FP64 in every mode)
  double* U;               // [nsub + npseudo][R][N]
  double* V;               // [nsub + npseudo][R][M]
  double* S;               // [nsub + npseudo][R][R]
  int* rank;               // [nsub + npseudo]
  int* tdim;               // [nsub] intermediate rank of the current stage
  int* rnew;               // [nsub] rank after truncation
  int* tmax;               // [nsub] largest t seen
  int* force;              // [2*nsub] t per advection stage, [2*nsub] r' ; -1 = rule
  int forced;
  unsigned* flags;         // [1]
  unsigned long long* clamps;  // [1]
  // scratch; the K-, L-step and V-hat working arrays (void*) hold FP64 in
  // DD_PREC_FP64 and FP32 in the mixed modes
  double* A;               // [nsub][MA][M]   weighted augmentation matrix
  double* Z;               // [nsub][MA][M]
  void* Qh;                // [nsub][T][M]    sqrt(w) * V-hat
  void* K1;                // [nsub][T][N]
  void* K2;                // [nsub][T][N]
  void* AL;                // [nsub][T][M]
  void* AL2;               // [nsub][T][M]
  double* K3;              // [nsub][T][N]    RK4: the K-step's initial value K0
  double* ghost;           // [nsub][2][T][face] RK4: frozen ghost rows (low, high face)
  double* gpart;           // [nsub][gpStride]
  double* small;           // [nsub][smallStride]
  double* rho;             // [3][ny*nx]: rho, jx, jy
  // inputs
  double* omx;             // [M]
  double* omy;             // [M]
  double* w;               // [M]
  double* sw;              // [M] sqrt(w)
  double* isw;             // [M] 1/sqrt(w)
  double* cs;              // [nsub][N] sigma_s in local order
  double* ct;              // [nsub][N] sigma_s + sigma_a
  double* Qsrc;            // [nsub][N]
  int nx;                  // global cells along x (moments)
  // small workspace offsets (doubles)
  int oRaccA, oCoef, oFill, oRinv, oRacc, oCp, oCn, oAm, oM0, oMm, oMp, oGLo, oGHi, oGLoN, oGHiN;
  int oEp, oEn, oOlo, oOhi, oTm, oGm, oGp, oBKlo, oBKhi, oS1, oS2, oP0, oPm, oPp, oBu, oBv;
  int oSig, oMv, oCrow, oGs, oGt, oQv, oW1, oW2, oW3, oW4, oW5, oW6, oRinvA, oSkip;
};

// The subdomain next to s along axis on side -1 / +1; at a physical face
// the layer slot of its prescribed inflow (slots after the subdomains: -x
// faces, +x, -y, +y, each by position along the face), or -1 (vacuum).
__host__ __device__ inline int neighbour(const Dev& d, int s, int axis, int side) {
  int sx = s % d.px, sy = s / d.px;
  if (axis == 0) {
    sx += side;
    if (sx < 0) return d.bc_in[0] ? d.nsub + sy : -1;
    if (sx >= d.px) return d.bc_in[1] ? d.nsub + d.py + sy : -1;
  } else {
    sy += side;
    if (sy < 0) return d.bc_in[2] ? d.nsub + 2 * d.py + sx : -1;
    if (sy >= d.py) return d.bc_in[3] ? d.nsub + 2 * d.py + d.px + sx : -1;
  }
  return sy * d.px + sx;
}

// local cell index of face entry f on a subdomain face
__device__ inline int face_cell(const Dev& d, int axis, bool high, int f) {
  if (axis == 0) return f * d.lnx + (high ? d.lnx - 1 : 0);
  return (high ? d.lny - 1 : 0) * d.lnx + f;
}

__device__ inline int face_len(const Dev& d, int axis) { return axis == 0 ? d.lny : d.lnx; }

__device__ inline int m0_of(const Dev& d, int s, int axis) {
  int lo = neighbour(d, s, axis, -1), hi = neighbour(d, s, axis, +1);
  return d.rank[s] + (lo >= 0 ? d.rank[lo] : 0) + (hi >= 0 ? d.rank[hi] : 0);
}

__device__ inline int dim_of(const Dev& d, int s, int axis, int which) {
  switch (which) {
    case DIM_M0: return m0_of(d, s, axis);
    case DIM_T: return d.tdim[s];
    case DIM_R: return d.rank[s];
    default: return d.rnew[s];
  }
}

__device__ inline double* small_of(const Dev& d, int s) { return d.small + (int64_t)s * d.smallStride; }
__device__ inline double* gpart_of(const Dev& d, int s) { return d.gpart + (int64_t)s * d.gpStride; }

// (i, j) with i <= j from the packed upper-triangle index k = j(j+1)/2 + i
__device__ inline void unpack_pair(int k, int& i, int& j) {
  int jj = (int)((sqrt(8.0 * k + 1.0) - 1.0) * 0.5);
  while (jj * (jj + 1) / 2 > k) --jj;
  while ((jj + 1) * (jj + 2) / 2 <= k) ++jj;
  j = jj;
  i = k - jj * (jj + 1) / 2;
}

// Order the LDS accesses of one wavefront around a point where its lanes
// exchange data through LDS (LDS operations of a wavefront complete in issue
// order; this keeps the compiler from moving them across the point).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// deterministic pseudo-random value in [-1, 1) (splitmix64 finaliser)
__device__ inline double hash_unit(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  x ^= x >> 31;
  return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

}  // namespace dd

// Launchers (host functions) implemented in the kernel translation units.
namespace dd {
// tall-skinny kernels
void init_kernels();
int ts_resident_wgs(const Dev& d);
void launch_aug_form(const Dev& d, int axis, int sd0, int nsd, hipStream_t st);
// Y = diag(rowscale) X B.  x64 / y64: X / Y is an FP64 array (else of the
// working type of the precision mode); exact: formed in FP64 whatever the
// precision mode (QR and SVD products).
void launch_gemm(const Dev& d, int axis, int sd0, int nsd, const void* X, bool x64, int64_t xsd, int rows,
                 int kdim, int ndim, int boff, int bld, void* Y, bool y64, int64_t ysd, const double* rowscale,
                 bool gram, int fill_off, bool rows_are_cells, bool exact, hipStream_t st, bool set_rank = false,
                 int skip_off = -1);
void launch_ang_reduce(const Dev& d, int axis, int sd0, int nsd, hipStream_t st);
void launch_kstep(const Dev& d, int axis, int sd0, int nsd, hipStream_t st);
void launch_spatial_reduce(const Dev& d, int axis, int sd0, int nsd, const void* Q, hipStream_t st);
void launch_lstep(const Dev& d, int axis, int sd0, int nsd, hipStream_t st);
void launch_coll_kstep(const Dev& d, int sd0, int nsd, hipStream_t st);
void launch_coll_reduce(const Dev& d, int sd0, int nsd, hipStream_t st);
void launch_coll_lstep(const Dev& d, int sd0, int nsd, hipStream_t st);
void launch_moments(const Dev& d, int nmom, hipStream_t st);
// moments with the per-subdomain vectors in smv (nsub x 3 x 64 doubles of
// device memory) and the cells written straight to rho, jx, jy (device)
void launch_moments_twopass(const Dev& d, int nmom, double* smv, double* rho, double* jx, double* jy,
                            hipStream_t st);
// small (one workgroup per subdomain) kernels
void launch_aug_svd(const Dev& d, int axis, int sd0, int nsd, hipStream_t st);
void launch_chol(const Dev& d, int axis, int sd0, int nsd, int ndim, int rows, int ngp, bool shift,
                 int acc_mode, double bscale, bool pivot, int oRinv, int oRacc, int ld, hipStream_t st, double* sout = nullptr,
                 int skip_mode = 0);
void launch_adv_prep(const Dev& d, int axis, int sd0, int nsd, hipStream_t st);
void launch_adv_sstep(const Dev& d, int axis, int sd0, int nsd, hipStream_t st);
void launch_trunc(const Dev& d, int axis, int sd0, int nsd, bool fold_rinv, hipStream_t st);
void launch_coll_prep(const Dev& d, int sd0, int nsd, hipStream_t st);
void launch_coll_sstep(const Dev& d, int sd0, int nsd, hipStream_t st);
}  // namespace dd
