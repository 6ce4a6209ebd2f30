// Host side of the DD-DLRA C ABI (include/dd_dlra.h): configuration checks,
// device arena layout, uploads, the launch plan of one time step
// (Algorithm 6: x stage, y stage, collision stage), hipGraph capture and the
// query calls.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "dd_dlra.h"
#include "dd_internal.h"
#include "dd_wide.h"

using dd::Dev;

struct dd_dlra_s {
  dd_dlra_config cfg;
  Dev d;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool own_ws = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::string err;
  // kernel timing (dd_dlra_profile)
  bool profiling = false;
  int prof_repeat = 1;
  std::vector<std::pair<hipGraph_t, hipGraphExec_t>> prof_graphs;  // replayed in profile mode
  bool capturing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct Pending {
    int kind, launches, reps;  // launches inside the event pair, of which reps repeat the phase
  };
  std::vector<Pending> pending;
  std::vector<int64_t> k_launch;
  std::vector<double> k_ms;
  double* noalloc_scratch = nullptr;  // device address of the static scratch on the handle's device
};

// Device scratch of dd_dlra_moments_noalloc: the per-subdomain moment
// vectors (up to 1024 subdomains x 3 moments x 64 ranks, 1.5 MiB), a
// file-scope array that each GPU the library runs on holds until the process
// ends.  Host code uses the per-device address from hipGetSymbolAddress,
// never the array's name (a host-side stand-in).
constexpr int NOALLOC_MAX_SUB = 1024;
constexpr size_t NOALLOC_DOUBLES = (size_t)NOALLOC_MAX_SUB * 3 * 64;
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace {

constexpr int MAX_DEVICES = 64;
double* g_scratch_ptr[MAX_DEVICES] = {};
std::once_flag g_scratch_once[MAX_DEVICES];
hipError_t g_scratch_err[MAX_DEVICES] = {};

// the device address of `scratch` on the current device (looked up once per
// device, with that device current); nullptr if the lookup failed
double* scratch_on_current_device(hipError_t* err) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
    *err = e != hipSuccess ? e : hipErrorInvalidDevice;
    return nullptr;
  }
  std::call_once(g_scratch_once[dev], [dev]() {
    void* p = nullptr;
    const hipError_t r = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[dev] = r;
    g_scratch_ptr[dev] = r == hipSuccess ? (double*)p : nullptr;
  });
  *err = g_scratch_err[dev];
  return g_scratch_ptr[dev];
}

}  // namespace

namespace {

thread_local std::string g_err;

enum Kind {
  K_AUG_FORM, K_GEMM_QR_A, K_AUG_SVD, K_GEMM_VHAT, K_CHOL, K_GEMM_QR_VHAT, K_ANG_REDUCE,
  K_ADV_PREP, K_KSTEP, K_GEMM_QR_K, K_SPATIAL_REDUCE, K_ADV_SSTEP, K_LSTEP, K_GEMM_QR_L, K_TRUNC,
  K_GEMM_FINAL_U, K_GEMM_FINAL_V, K_COLL_PREP, K_COLL_KSTEP, K_COLL_REDUCE, K_COLL_SSTEP,
  K_COLL_LSTEP, K_GEMM_QR_KC, K_GEMM_QR_LC, K_GEMM_QR_K_IP, K_GEMM_QR_L_IP, K_GEMM_QR_KC_IP, K_GEMM_QR_LC_IP,
  K_W_GRAM_A, K_W_GRAM_VHAT, K_W_ANG, K_W_GRAM_K, K_W_SPATIAL, K_W_GRAM_L, K_W_GRAM_KC, K_W_COLL_REDUCE,
  K_W_CHOL, K_W_RK_PREP, K_GEMM_K0, K_W_RK_KSTEP,
  K_COUNT
};

const char* const kKindName[K_COUNT] = {
  "k_aug_form", "k_gemm[QR A]", "s_aug_svd", "k_gemm[V-hat=A*Coef]", "s_chol",
  "k_gemm[QR V-hat]", "k_ang_reduce", "s_adv_prep", "k_kstep", "k_gemm[QR K1]", "k_spatial_reduce",
  "s_adv_sstep", "k_lstep", "k_gemm[QR L1]", "s_trunc", "k_gemm[U=Q*Bu]", "k_gemm[V=QL*Bv]",
  "s_coll_prep", "k_coll_kstep", "k_coll_reduce", "s_coll_sstep", "k_coll_lstep",
  "k_gemm[QR K1 collision]", "k_gemm[QR L1 collision]", "k_gemm[QR K1 in place]", "k_gemm[QR L1 in place]",
  "k_gemm[QR K1 collision in place]", "k_gemm[QR L1 collision in place]",
  "kw_xgram[Gram A]", "kw_xgram[Gram V-hat]", "kw_xgram[angular]", "kw_xgram[Gram K1]", "kw_xgram[spatial]",
  "kw_xgram[Gram L1]", "kw_xgram[Gram K1 collision]", "kw_xgram[collision]", "sw_chol",
  "sw_rk_prep", "k_gemm[K0=U*Am]", "kw_rk_kstep",
};

struct Layout {
  int wide;
  int R, T, MA, N, M, nsub, ntN, ntM, nwgN, nwgM, gpTile;
  int64_t gpStride, smallStride;
  int off[48];
  size_t bytes;
  // byte offsets of the arena segments
  size_t oU, oV, oS, oA, oZ, oQh, oK1, oK2, oAL, oAL2, oGP, oSM, oRho, oIn, oCs, oCt, oQ, oInt, oFlags;
  size_t oK3, oGhost;  // RK4 only: the K-step's initial value and the frozen ghost rows
  int npseudo;         // layer slots of the inflow faces
  int face;            // cells on the longer subdomain face
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// Validate everything that does not need the initial factors.  Returns an
// empty string on success.
std::string validate(const dd_dlra_config* c) {
  if (!c) return "config is NULL";
  if (c->nx <= 0 || c->ny <= 0 || c->px <= 0 || c->py <= 0) return "grid and subdomain counts must be positive";
  if (c->nx % c->px || c->ny % c->py) return "nx must be divisible by px and ny by py";
  if (!(c->x1 > c->x0) || !(c->y1 > c->y0)) return "empty domain";
  const double hx = (c->x1 - c->x0) / c->nx, hy = (c->y1 - c->y0) / c->ny;
  if (fabs(hx - hy) > 1e-12 * hx) return "cells must be square: (x1-x0)/nx != (y1-y0)/ny";
  if (c->n_dir <= 0) return "n_dir must be positive";
  if (!c->omega_x || !c->omega_y || !c->w) return "direction arrays must not be NULL";
  if (!c->sigma_s || !c->sigma_a || !c->Q) return "field arrays must not be NULL";
  const size_t M = c->n_dir, n = (size_t)c->nx * c->ny;
  if (!finite_all(c->omega_x, M) || !finite_all(c->omega_y, M) || !finite_all(c->w, M))
    return "non-finite direction data";
  for (size_t q = 0; q < M; ++q)
    if (!(c->w[q] > 0.0)) return "quadrature weights must be positive";
  if (!finite_all(c->sigma_s, n) || !finite_all(c->sigma_a, n) || !finite_all(c->Q, n)) return "non-finite field data";
  for (size_t p = 0; p < n; ++p)
    if (c->sigma_s[p] < 0.0 || c->sigma_a[p] < 0.0) return "cross sections must be non-negative";
  if (!(c->dt > 0.0) || !std::isfinite(c->dt)) return "dt must be positive";
  if (!(c->c_adv >= 0.0) || !std::isfinite(c->c_adv)) return "c_adv must be non-negative";
  if (c->rank_mode != DD_RANK_FIXED && c->rank_mode != DD_RANK_ADAPTIVE) return "unknown rank_mode";
  if (c->rank_mode == DD_RANK_FIXED && c->r_fixed < 1) return "r_fixed must be >= 1";
  if (c->rank_mode == DD_RANK_ADAPTIVE) {
    if (c->r_min < 1 || c->r_max < c->r_min) return "need 1 <= r_min <= r_max";
    if (!(c->tol >= 0.0)) return "tol must be >= 0";
  }
  if (!(c->tol_aug_rel >= 0.0)) return "tol_aug_rel must be >= 0";
  const int R = c->rank_mode == DD_RANK_FIXED ? c->r_fixed : c->r_max;
  if (c->r_int_max < R) return "r_int_max must be at least the stored-rank capacity";
  if (c->r_int_max > dd::WCAP_T) return "r_int_max beyond the supported maximum of 128";
  if (R > dd::WCAP_R) return "stored-rank capacity beyond the supported maximum of 64";
  if (c->integrator != DD_INT_EULER && c->integrator != DD_INT_RK4) return "unknown integrator";
  if (c->integrator == DD_INT_RK4 && c->precision != DD_PREC_FP64)
    return "RK4 substeps run in DD_PREC_FP64 only";
  if (c->precision < DD_PREC_FP64 || c->precision > DD_PREC_MIXED_BF16) return "unknown precision";
  if (c->exec_mode < DD_EXEC_PER_SUBDOMAIN || c->exec_mode > DD_EXEC_BATCHED_GRAPH) return "unknown exec_mode";
  for (int f = 0; f < 4; ++f) {
    if (c->bc[f] == DD_BC_VACUUM) continue;
    if (c->bc[f] != DD_BC_INFLOW_LOWRANK) return "unknown boundary condition of face " + std::to_string(f);
    if (c->bc_rank[f] < 1 || c->bc_rank[f] > R)
      return "inflow rank of face " + std::to_string(f) + " must be between 1 and the stored-rank capacity";
    if (!c->bc_a[f] || !c->bc_b[f]) return "inflow arrays of face " + std::to_string(f) + " must not be NULL";
    const size_t nf = f < 2 ? c->ny : c->nx;
    if (!finite_all(c->bc_a[f], nf * c->bc_rank[f]) || !finite_all(c->bc_b[f], M * c->bc_rank[f]))
      return "non-finite inflow data of face " + std::to_string(f);
  }
  return "";
}

// The narrow plan's kernels hold up to 48 intermediate and 64 augmentation
// columns (stored ranks up to 21; its 64-column row reductions would spill
// registers); larger capacities take the wide plan.
// DD_DLRA_PLAN=wide in the environment selects the wide plan for any
// capacity (used to test it on small problems).
bool wide_plan(const dd_dlra_config* c) {
  const int R = c->rank_mode == DD_RANK_FIXED ? c->r_fixed : c->r_max;
  const char* env = getenv("DD_DLRA_PLAN");
  if (env && strcmp(env, "wide") == 0) return true;
  if (c->integrator == DD_INT_RK4) return true;  // the RK4 substeps exist in the wide kernels
  return c->r_int_max > 48 || 3 * R > dd::CAP;
}

Layout make_layout(const dd_dlra_config* c) {
  Layout L;
  L.wide = wide_plan(c) ? 1 : 0;
  L.R = c->rank_mode == DD_RANK_FIXED ? c->r_fixed : c->r_max;
  L.T = c->r_int_max;
  L.MA = 3 * L.R;
  L.nsub = c->px * c->py;
  L.N = (c->nx / c->px) * (c->ny / c->py);
  L.M = c->n_dir;
  L.ntN = (L.N + dd::TILE - 1) / dd::TILE;
  L.ntM = (L.M + dd::TILE - 1) / dd::TILE;
  // room for partial sums of up to this many workgroups per subdomain (the
  // grid actually used is chosen at creation from the kernels' occupancy)
  const int cap = std::min(64, std::max(1, (4096 + L.nsub - 1) / L.nsub));
  L.nwgN = std::min(L.ntN, cap);
  L.nwgM = std::min(L.ntM, cap);
  const int R = L.R, T = L.T, MA = L.MA;
  L.gpTile = std::max(std::max(MA * MA, 3 * T * T + 3 * R * T), std::max(2 * T * T + 4 * T * R, 2 * R * R + R));
  L.gpStride = (int64_t)std::max(L.nwgN, L.nwgM) * L.gpTile;
  // small workspace
  int o = 0;
  int* f = L.off;
  auto take = [&](int n) {
    int r = o;
    o += (n + 31) & ~31;
    return r;
  };
  int k = 0;
  f[k++] = take(MA * MA);  // RaccA (Cholesky-QR factor of the augmentation matrix)
  f[k++] = take(MA * T);   // Coef
  f[k++] = take(std::max(T, MA));  // Fill
  f[k++] = take(T * T);    // Rinv
  f[k++] = take(T * T);    // Racc
  f[k++] = take(T * T);    // Cp
  f[k++] = take(T * T);    // Cn
  f[k++] = take(R * T);    // Am
  for (int i = 0; i < 7; ++i) f[k++] = take(R * T);  // M0 Mm Mp GLo GHi GLoN GHiN
  f[k++] = take(T * T);    // Ep
  f[k++] = take(T * T);    // En
  f[k++] = take(R * T);    // Olo
  f[k++] = take(R * T);    // Ohi
  f[k++] = take(R * T);    // Tm
  f[k++] = take(T * T);    // Gm
  f[k++] = take(T * T);    // Gp
  f[k++] = take(T * T);    // BKlo
  f[k++] = take(T * T);    // BKhi
  f[k++] = take(T * T);    // S1
  f[k++] = take(T * T);    // S2
  f[k++] = take(T * T);    // P0
  f[k++] = take(T * T);    // Pm
  f[k++] = take(T * T);    // Pp
  f[k++] = take(T * T);    // Bu
  f[k++] = take(T * T);    // Bv
  f[k++] = take(MA);       // Sig
  f[k++] = take(R);        // Mv
  f[k++] = take(R);        // Crow
  f[k++] = take(R * R);    // Gs
  f[k++] = take(R * R);    // Gt
  f[k++] = take(R);        // Qv
  for (int i = 0; i < 6; ++i) f[k++] = take(T * T);  // W1..W6
  f[k++] = take(MA * MA);  // RinvA
  f[k++] = take(1);        // Skip (the last Cholesky-QR pass may be skipped)
  L.smallStride = o;
  // arena
  const size_t d8 = sizeof(double);
  // K-, L-step and V-hat working arrays: FP32 in the mixed modes
  const size_t es = c->precision == DD_PREC_FP64 ? sizeof(double) : sizeof(float);
  const size_t ns = L.nsub;
  size_t b = 0;
  auto seg = [&](size_t bytes) {
    size_t r = b;
    b = align256(b + bytes);
    return r;
  };
  // inflow faces act as neighbours held in extra "layer" slots after the
  // subdomains (-x: py, +x: py, -y: px, +y: px), in the state arrays only
  L.npseudo = 0;
  for (int f = 0; f < 4; ++f)
    if (c->bc[f] == DD_BC_INFLOW_LOWRANK) L.npseudo = 2 * (c->px + c->py);
  const size_t nsx = ns + L.npseudo;
  L.oU = seg(nsx * L.N * R * d8);
  L.oV = seg(nsx * L.M * R * d8);
  L.oS = seg(nsx * R * R * d8);
  L.oA = seg(ns * L.M * MA * d8);
  L.oZ = seg(ns * L.M * std::max(MA, T) * d8);  // the wide plan's second V-hat buffer
  L.oQh = seg(ns * L.M * T * es);
  L.oK1 = seg(ns * L.N * T * es);
  L.oK2 = seg(ns * L.N * T * es);
  L.oAL = seg(ns * L.M * T * es);
  L.oAL2 = seg(ns * L.M * T * es);
  L.oGP = seg(ns * L.gpStride * d8);
  L.oSM = seg(ns * L.smallStride * d8);
  L.oRho = seg(3 * (size_t)c->nx * c->ny * d8);
  L.oIn = seg(5 * (size_t)L.M * d8);
  L.oCs = seg(ns * L.N * d8);
  L.oCt = seg(ns * L.N * d8);
  L.oQ = seg(ns * L.N * d8);
  L.oInt = seg((8 * ns + L.npseudo) * sizeof(int));
  L.oFlags = seg(64);
  L.face = std::max(c->nx / c->px, c->ny / c->py);
  L.oK3 = L.oGhost = 0;
  if (c->integrator == DD_INT_RK4) {
    L.oK3 = seg(ns * L.N * T * d8);
    L.oGhost = seg(ns * 2 * (size_t)T * L.face * d8);
  }
  L.bytes = b;
  return L;
}

// The wide plan's reductions read by wide kernels use twice the workgroups
// per subdomain of the other tall-skinny kernels (up to the room for
// partial sums): their launch length is set by the few high-rank
// subdomains, which then spread over more compute units.
void set_wide_partials(Dev& d) {
  const int capN = std::max(1, (int)(d.gpStride / d.gpTile));
  d.xpN = std::min(2 * d.nwgN, capN);
  d.xpM = std::min(2 * d.nwgM, capN);
  // the Galerkin job sets (several blocks per subdomain) and the Gram of
  // the augmentation matrix are summed by one workgroup of the preparation
  // and SVD kernels: at most 8 row splits
  d.xgN = std::min(d.xpN, 8);
  d.xgM = std::min(d.xpM, 8);
}


void fill_dev(Dev& d, const Layout& L, const dd_dlra_config* c, char* base) {
  memset(&d, 0, sizeof(d));
  d.px = c->px;
  d.py = c->py;
  d.lnx = c->nx / c->px;
  d.lny = c->ny / c->py;
  d.N = L.N;
  d.M = L.M;
  d.nsub = L.nsub;
  d.nx = c->nx;
  d.h = (c->x1 - c->x0) / c->nx;
  d.dt = c->dt;
  d.c = c->c_adv;
  double W = 0.0;
  for (int q = 0; q < c->n_dir; ++q) W += c->w[q];
  d.W = W;
  d.R = L.R;
  d.T = L.T;
  d.MA = L.MA;
  d.ntN = L.ntN;
  d.ntM = L.ntM;
  d.nwgN = L.nwgN;
  d.nwgM = L.nwgM;
  d.gpTile = L.gpTile;
  d.gpStride = L.gpStride;
  set_wide_partials(d);
  d.smallStride = L.smallStride;
  d.rank_mode = c->rank_mode;
  d.r_fixed = c->r_fixed;
  d.r_min = c->rank_mode == DD_RANK_FIXED ? c->r_fixed : c->r_min;
  d.r_max = c->rank_mode == DD_RANK_FIXED ? c->r_fixed : c->r_max;
  d.r_int_max = c->r_int_max;
  d.strict = c->strict_caps;
  d.prec = c->precision;
  d.wide = L.wide;
  d.rk4 = c->integrator == DD_INT_RK4 ? 1 : 0;
  d.face = L.face;
  d.K3 = d.rk4 ? (double*)(base + L.oK3) : nullptr;
  d.ghost = d.rk4 ? (double*)(base + L.oGhost) : nullptr;
  d.tol = c->tol;
  d.tol_aug_rel = c->tol_aug_rel;
  d.U = (double*)(base + L.oU);
  d.V = (double*)(base + L.oV);
  d.S = (double*)(base + L.oS);
  d.A = (double*)(base + L.oA);
  d.Z = (double*)(base + L.oZ);
  d.Qh = (void*)(base + L.oQh);
  d.K1 = (void*)(base + L.oK1);
  d.K2 = (void*)(base + L.oK2);
  d.AL = (void*)(base + L.oAL);
  d.AL2 = (void*)(base + L.oAL2);
  d.gpart = (double*)(base + L.oGP);
  d.small = (double*)(base + L.oSM);
  d.rho = (double*)(base + L.oRho);
  double* in = (double*)(base + L.oIn);
  d.omx = in;
  d.omy = in + L.M;
  d.w = in + 2 * L.M;
  d.sw = in + 3 * L.M;
  d.isw = in + 4 * L.M;
  d.cs = (double*)(base + L.oCs);
  d.ct = (double*)(base + L.oCt);
  d.Qsrc = (double*)(base + L.oQ);
  int* ip = (int*)(base + L.oInt);
  d.rank = ip;  // [nsub + npseudo]
  d.tdim = ip + L.nsub + L.npseudo;
  d.rnew = d.tdim + L.nsub;
  d.tmax = d.rnew + L.nsub;
  d.force = d.tmax + L.nsub;
  d.npseudo = L.npseudo;
  for (int f = 0; f < 4; ++f) d.bc_in[f] = c->bc[f] == DD_BC_INFLOW_LOWRANK ? 1 : 0;
  d.flags = (unsigned*)(base + L.oFlags);
  d.clamps = (unsigned long long*)(base + L.oFlags + 8);
  const int* f = L.off;
  int k = 0;
  d.oRaccA = f[k++]; d.oCoef = f[k++]; d.oFill = f[k++]; d.oRinv = f[k++]; d.oRacc = f[k++];
  d.oCp = f[k++]; d.oCn = f[k++]; d.oAm = f[k++];
  d.oM0 = f[k++]; d.oMm = f[k++]; d.oMp = f[k++]; d.oGLo = f[k++]; d.oGHi = f[k++]; d.oGLoN = f[k++]; d.oGHiN = f[k++];
  d.oEp = f[k++]; d.oEn = f[k++]; d.oOlo = f[k++]; d.oOhi = f[k++]; d.oTm = f[k++];
  d.oGm = f[k++]; d.oGp = f[k++]; d.oBKlo = f[k++]; d.oBKhi = f[k++]; d.oS1 = f[k++]; d.oS2 = f[k++];
  d.oP0 = f[k++]; d.oPm = f[k++]; d.oPp = f[k++]; d.oBu = f[k++]; d.oBv = f[k++];
  d.oSig = f[k++]; d.oMv = f[k++]; d.oCrow = f[k++]; d.oGs = f[k++]; d.oGt = f[k++]; d.oQv = f[k++];
  d.oW1 = f[k++]; d.oW2 = f[k++]; d.oW3 = f[k++]; d.oW4 = f[k++]; d.oW5 = f[k++]; d.oW6 = f[k++];
  d.oRinvA = f[k++];
  d.oSkip = f[k++];
}

std::string check_factors(const dd_dlra_config* c, const Layout& L, const int32_t* rank, const double* const* U,
                          const double* const* S, const double* const* V) {
  if (!rank || !U || !S || !V) return "initial factor arrays must not be NULL";
  const double h = (c->x1 - c->x0) / c->nx;
  for (int s = 0; s < L.nsub; ++s) {
    const int r = rank[s];
    if (r < 1 || r > L.R) return "initial rank of subdomain " + std::to_string(s) + " outside [1, capacity]";
    if (!U[s] || !S[s] || !V[s]) return "NULL factor of subdomain " + std::to_string(s);
    if (!finite_all(U[s], (size_t)L.N * r) || !finite_all(S[s], (size_t)r * r) || !finite_all(V[s], (size_t)L.M * r))
      return "non-finite initial factor in subdomain " + std::to_string(s);
    for (int i = 0; i < r; ++i)
      for (int j = 0; j <= i; ++j) {
        double gu = 0.0, gv = 0.0;
        for (int p = 0; p < L.N; ++p) gu += U[s][(size_t)i * L.N + p] * U[s][(size_t)j * L.N + p];
        for (int q = 0; q < L.M; ++q) gv += V[s][(size_t)i * L.M + q] * c->w[q] * V[s][(size_t)j * L.M + q];
        gu *= h * h;
        const double e = (i == j) ? 1.0 : 0.0;
        if (fabs(gu - e) > 1e-8 || fabs(gv - e) > 1e-8)
          return "initial factors of subdomain " + std::to_string(s) +
                 " are not orthonormal (need h^2 U^T U = I and V^T diag(w) V = I)";
      }
  }
  return "";
}

#define HIPCHK(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) {                                                          \
      h->err = std::string(#call) + ": " + hipGetErrorString(e_);                    \
      return DD_EHIP;                                                                \
    }                                                                                \
  } while (0)

dd_status upload_factors(dd_dlra_handle h, const int32_t* rank, const double* const* U, const double* const* S,
                         const double* const* V) {
  const Dev& d = h->d;
  std::vector<double> buf;
  for (int s = 0; s < d.nsub; ++s) {
    const int r = rank[s];
    buf.assign((size_t)d.N * d.R, 0.0);
    memcpy(buf.data(), U[s], sizeof(double) * (size_t)d.N * r);
    HIPCHK(hipMemcpyAsync(d.U + (size_t)s * d.N * d.R, buf.data(), buf.size() * 8, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    buf.assign((size_t)d.M * d.R, 0.0);
    memcpy(buf.data(), V[s], sizeof(double) * (size_t)d.M * r);
    HIPCHK(hipMemcpyAsync(d.V + (size_t)s * d.M * d.R, buf.data(), buf.size() * 8, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    buf.assign((size_t)d.R * d.R, 0.0);
    for (int j = 0; j < r; ++j)
      for (int i = 0; i < r; ++i) buf[i + (size_t)j * d.R] = S[s][i + (size_t)j * r];
    HIPCHK(hipMemcpyAsync(d.S + (size_t)s * d.R * d.R, buf.data(), buf.size() * 8, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  std::vector<int> iv(d.nsub);
  for (int s = 0; s < d.nsub; ++s) iv[s] = rank[s];
  HIPCHK(hipMemcpyAsync(d.rank, iv.data(), d.nsub * sizeof(int), hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(d.tmax, iv.data(), d.nsub * sizeof(int), hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return DD_OK;
}

// The layer slots of the inflow faces: for each subdomain along an inflow
// face, the thin QR a_s = Q_a R_a (classical Gram-Schmidt applied twice) of
// its part of the face profile gives U = Q_a / h on the layer's cells next
// to the subdomain, S = h R_a and V = b (Section 4's prescribed inflow as a
// neighbour; see the header).
dd_status upload_inflow_layers(dd_dlra_handle h, const dd_dlra_config* c) {
  const Dev& d = h->d;
  if (d.npseudo == 0) return DD_OK;
  const int N = d.N, M = d.M, R = d.R;
  for (int f = 0; f < 4; ++f) {
    if (!d.bc_in[f]) continue;
    const int rb = c->bc_rank[f];
    const int axis = f < 2 ? 0 : 1;
    const bool layer_high = (f % 2) == 0;  // a low face's layer touches the subdomain with its high face
    const int nface = axis == 0 ? d.lny : d.lnx;       // cells along one subdomain's face
    const int ntot = axis == 0 ? c->ny : c->nx;        // along the whole face
    const int npos = axis == 0 ? d.py : d.px;
    const int slot0 = d.nsub + (f == 0 ? 0 : f == 1 ? d.py : f == 2 ? 2 * d.py : 2 * d.py + d.px);
    for (int j = 0; j < npos; ++j) {
      std::vector<double> Q((size_t)nface * rb), Rm((size_t)rb * rb, 0.0);
      for (int k = 0; k < rb; ++k)
        for (int i = 0; i < nface; ++i) Q[i + (size_t)k * nface] = c->bc_a[f][(size_t)k * ntot + j * nface + i];
      for (int k = 0; k < rb; ++k) {
        double* q = &Q[(size_t)k * nface];
        const double n0 = sqrt(std::inner_product(q, q + nface, q, 0.0));
        for (int pass = 0; pass < 2; ++pass)
          for (int l = 0; l < k; ++l) {
            const double* p = &Q[(size_t)l * nface];
            const double dot = std::inner_product(p, p + nface, q, 0.0);
            Rm[l + (size_t)k * rb] += dot;
            for (int i = 0; i < nface; ++i) q[i] -= dot * p[i];
          }
        const double nrm = sqrt(std::inner_product(q, q + nface, q, 0.0));
        if (nrm > 1e-14 * n0 && nrm > 0.0) {
          Rm[k + (size_t)k * rb] = nrm;
          for (int i = 0; i < nface; ++i) q[i] /= nrm;
        } else {
          for (int i = 0; i < nface; ++i) q[i] = 0.0;  // dependent: a zero column, a zero row of R
        }
      }
      std::vector<double> U((size_t)N * R, 0.0), Sv((size_t)R * R, 0.0), V((size_t)M * R, 0.0);
      for (int k = 0; k < rb; ++k) {
        for (int i = 0; i < nface; ++i) {
          const int cell = axis == 0 ? i * d.lnx + (layer_high ? d.lnx - 1 : 0)
                                     : (layer_high ? d.lny - 1 : 0) * d.lnx + i;
          U[(size_t)k * N + cell] = Q[i + (size_t)k * nface] / d.h;
        }
        for (int q = 0; q < M; ++q) V[(size_t)k * M + q] = c->bc_b[f][(size_t)k * M + q];
        for (int l = 0; l < rb; ++l) Sv[l + (size_t)k * R] = d.h * Rm[l + (size_t)k * rb];
      }
      const int slot = slot0 + j;
      HIPCHK(hipMemcpy(d.U + (size_t)slot * N * R, U.data(), U.size() * 8, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(d.V + (size_t)slot * M * R, V.data(), V.size() * 8, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(d.S + (size_t)slot * R * R, Sv.data(), Sv.size() * 8, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(d.rank + slot, &rb, sizeof(int), hipMemcpyHostToDevice));
    }
  }
  return DD_OK;
}

// ---------------------------------------------------------------- launch plan

hipEvent_t next_event(dd_dlra_handle h) {
  if (h->ev_used == h->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->ev_pool.push_back(e);
  }
  return h->ev_pool[h->ev_used++];
}

// Run one phase either for all subdomains in one launch (batched modes) or
// once per subdomain (the plain per-subdomain mode); with profiling on (and
// not capturing a graph) the phase is bracketed by a pair of events.
// Phases whose launch reads one set of buffers and overwrites another, so
// that launching them again leaves the same result (the in-place Cholesky-QR
// passes and the small kernels are not).
bool repeatable(int kind) {
  switch (kind) {
    case K_AUG_FORM: case K_GEMM_VHAT: case K_ANG_REDUCE: case K_KSTEP: case K_GEMM_QR_K:
    case K_SPATIAL_REDUCE: case K_LSTEP: case K_GEMM_QR_L: case K_GEMM_FINAL_U: case K_GEMM_FINAL_V:
    case K_COLL_KSTEP: case K_COLL_REDUCE: case K_COLL_LSTEP: case K_GEMM_QR_KC: case K_GEMM_QR_LC:
    case K_W_GRAM_A: case K_W_GRAM_VHAT: case K_W_ANG: case K_W_GRAM_K: case K_W_SPATIAL: case K_W_GRAM_L:
    case K_W_GRAM_KC: case K_W_COLL_REDUCE: case K_W_RK_PREP: case K_GEMM_K0: case K_W_RK_KSTEP:
      return true;
    default:
      return false;
  }
}

template <class F>
void phase(dd_dlra_handle h, int kind, F&& f) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool timed = h->profiling && !h->capturing && h->ev_used + 2 <= 1u << 16;
  if (timed) {
    e0 = next_event(h);
    e1 = next_event(h);
    if (e0 && e1) (void)hipEventRecord(e0, h->stream);
  }
  // with profiling at repeat > 1, an idempotent tall-skinny phase is
  // captured repeat times into a graph that is replayed inside the event
  // pair: back-to-back graph nodes carry little dispatch overhead, so the
  // average comes close to the kernel's own duration
  const int reps = (timed && repeatable(kind)) ? h->prof_repeat : 1;
  int launches = 0;
  auto launch_all = [&]() {
    for (int rep = 0; rep < reps; ++rep) {
      if (h->cfg.exec_mode == DD_EXEC_PER_SUBDOMAIN) {
        for (int s = 0; s < h->d.nsub; ++s) f(s, 1);
        launches += h->d.nsub;
      } else {
        f(0, h->d.nsub);
        launches += 1;
      }
    }
  };
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  if (reps > 1 && hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
    launch_all();
    if (hipStreamEndCapture(h->stream, &g) != hipSuccess ||
        hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      g = nullptr;
      ge = nullptr;
    }
  }
  if (ge) {
    // the capture recorded no work: restart the pair around the replay
    if (e0) (void)hipEventRecord(e0, h->stream);
    (void)hipGraphLaunch(ge, h->stream);
    h->prof_graphs.push_back({g, ge});
  } else if (reps > 1) {
    launches = 0;
    launch_all();
  } else {
    launch_all();
  }
  if (timed && e0 && e1) {
    (void)hipEventRecord(e1, h->stream);
    h->pending.push_back({kind, launches, reps});
  }
}

// Shifted Cholesky QR with three passes on X (rows x n; n = dim of kind
// ndim) leaving Q in Y: the first pass reads X and writes Y, the second and
// third work on Y in place (each strip of rows is read completely before it
// is written); the R factors accumulate in the small workspace.  When the
// second pass takes the near-identity factor (its Gram within 1e-3 of the
// identity), its output is already orthonormal to rounding: the third
// Cholesky pass then takes R = I and its in-place product exits at once.  With final_dst set, the last
// product writes there instead (stride final_sd, optional row scale, Rinv
// scaled by bscale); with s_dst set, the last Cholesky pass also stores
// Racc^T there as the coefficient matrix of each subdomain.  With
// defer_last, the last product is left to the caller: Q = Y Rinv with Rinv
// in the small workspace.
void chol_qr3(dd_dlra_handle h, int axis, int ndim, void* X, void* Y, int64_t sdstride, int rows, bool cells,
              double* final_dst, int64_t final_sd, const double* final_rowscale, double bscale, int gemm_kind,
              int ip_kind, double* s_dst = nullptr, bool defer_last = false) {
  const Dev& d = h->d;
  hipStream_t st = h->stream;
  const int ngp = cells ? d.nwgN : d.nwgM;
  phase(h, K_CHOL, [&](int s0, int ns) {
    dd::launch_chol(d, axis, s0, ns, ndim, rows, ngp, true, 1, 1.0, false, d.oRinv, d.oRacc, d.T, st);
  });
  phase(h, gemm_kind, [&](int s0, int ns) {
    dd::launch_gemm(d, axis, s0, ns, X, false, sdstride, rows, ndim, ndim, d.oRinv, d.T, Y, false, sdstride, nullptr,
                    true, d.oFill, cells, true, st);
  });
  phase(h, K_CHOL, [&](int s0, int ns) {
    dd::launch_chol(d, axis, s0, ns, ndim, rows, ngp, false, 2, 1.0, false, d.oRinv, d.oRacc, d.T, st, nullptr, 1);
  });
  phase(h, ip_kind, [&](int s0, int ns) {
    dd::launch_gemm(d, axis, s0, ns, Y, false, sdstride, rows, ndim, ndim, d.oRinv, d.T, Y, false, sdstride, nullptr,
                    true, d.oFill, cells, true, st);
  });
  phase(h, K_CHOL, [&](int s0, int ns) {
    dd::launch_chol(d, axis, s0, ns, ndim, rows, ngp, false, 2, bscale, false, d.oRinv, d.oRacc, d.T, st, s_dst, 2);
  });
  if (defer_last) return;
  void* dst = final_dst ? (void*)final_dst : Y;
  const int64_t dsd = final_dst ? final_sd : sdstride;
  phase(h, final_dst ? gemm_kind : ip_kind, [&](int s0, int ns) {
    dd::launch_gemm(d, axis, s0, ns, Y, false, sdstride, rows, ndim, ndim, d.oRinv, d.T, dst, final_dst != nullptr,
                    dsd, final_rowscale, false, d.oFill, cells, true, st, false, final_dst ? -1 : d.oSkip);
  });
}

void enqueue_advection(dd_dlra_handle h, int axis, int upto = 0) {
  const Dev& d = h->d;
  hipStream_t st = h->stream;
  const int64_t sdMA = (int64_t)d.M * d.MA, sdMT = (int64_t)d.M * d.T, sdNT = (int64_t)d.N * d.T;
  // Algorithm 4: augmentation.  A = sqrt(w) L0 = Q RaccA by three passes of
  // shifted Cholesky QR (the first one pivoted; Q itself is not kept), then
  // the SVD of the small factor and V-hat = A B Sigma^-2.
  phase(h, K_AUG_FORM, [&](int s0, int ns) { dd::launch_aug_form(d, axis, s0, ns, st); });
  for (int pass = 0; pass < 3; ++pass) {
    phase(h, K_CHOL, [&](int s0, int ns) {
      dd::launch_chol(d, axis, s0, ns, dd::DIM_M0, d.M, d.nwgM, pass == 0, pass == 0 ? 1 : 2, 1.0, pass == 0,
                      d.oRinvA, d.oRaccA, d.MA, st, nullptr, pass);
    });
    if (pass == 2) break;
    // pass 0: Z = A P R^-1; pass 1: Z <- Z R^-1 in place (each strip of rows
    // is read completely before it is written)
    phase(h, K_GEMM_QR_A, [&](int s0, int ns) {
      dd::launch_gemm(d, axis, s0, ns, pass == 0 ? d.A : d.Z, true, sdMA, d.M, dd::DIM_M0, dd::DIM_M0, d.oRinvA,
                      d.MA, d.Z, true, sdMA, nullptr, true, d.oFill, false, true, st);
    });
  }
  phase(h, K_AUG_SVD, [&](int s0, int ns) { dd::launch_aug_svd(d, axis, s0, ns, st); });
  phase(h, K_GEMM_VHAT, [&](int s0, int ns) {
    dd::launch_gemm(d, axis, s0, ns, d.A, true, sdMA, d.M, dd::DIM_M0, dd::DIM_T, d.oCoef, d.MA, d.Qh, false, sdMT,
                    nullptr, true, d.oFill, false, true, st);
  });
  // two Cholesky QR passes in place make V-hat orthonormal to working
  // precision (the second is skipped when the first took the near-identity
  // factor)
  for (int pass = 0; pass < 2; ++pass) {
    phase(h, K_CHOL, [&](int s0, int ns) {
      dd::launch_chol(d, axis, s0, ns, dd::DIM_T, d.M, d.nwgM, false, 0, 1.0, false, d.oRinv, d.oRacc, d.T, st,
                      nullptr, pass + 1);
    });
    phase(h, K_GEMM_QR_VHAT, [&](int s0, int ns) {
      dd::launch_gemm(d, axis, s0, ns, d.Qh, false, sdMT, d.M, dd::DIM_T, dd::DIM_T, d.oRinv, d.T, d.Qh, false, sdMT,
                      nullptr, pass == 0, d.oFill, false, true, st, false, pass == 1 ? d.oSkip : -1);
    });
  }
  if (upto == DD_PROBE_VHAT) return;
  // angular Galerkin matrices, eigen-split of C, K-step coefficients
  phase(h, K_ANG_REDUCE, [&](int s0, int ns) { dd::launch_ang_reduce(d, axis, s0, ns, st); });
  phase(h, K_ADV_PREP, [&](int s0, int ns) { dd::launch_adv_prep(d, axis, s0, ns, st); });
  // Algorithm 1/2 steps 1-2: K-step, QR
  phase(h, K_KSTEP, [&](int s0, int ns) { dd::launch_kstep(d, axis, s0, ns, st); });
  if (upto == DD_PROBE_K1) return;
  chol_qr3(h, axis, dd::DIM_T, d.K1, d.K2, sdNT, d.N, true, nullptr, 0, nullptr, 1.0, K_GEMM_QR_K, K_GEMM_QR_K_IP);
  if (upto == DD_PROBE_U1) return;
  // step 3: S-step
  phase(h, K_SPATIAL_REDUCE, [&](int s0, int ns) { dd::launch_spatial_reduce(d, axis, s0, ns, d.K2, st); });
  phase(h, K_ADV_SSTEP, [&](int s0, int ns) { dd::launch_adv_sstep(d, axis, s0, ns, st); });
  if (upto == DD_PROBE_S2) return;
  // steps 4-5: L-step, weighted QR
  phase(h, K_LSTEP, [&](int s0, int ns) { dd::launch_lstep(d, axis, s0, ns, st); });
  if (upto == DD_PROBE_L1) return;
  // (the last product, Q_L = Y Rinv, is folded into the final V product)
  chol_qr3(h, axis, dd::DIM_T, d.AL, d.AL2, sdMT, d.M, false, nullptr, 0, nullptr, 1.0, K_GEMM_QR_L, K_GEMM_QR_L_IP,
           nullptr, true);
  // Algorithm 5: truncation, then rotate the bases into the state
  phase(h, K_TRUNC, [&](int s0, int ns) { dd::launch_trunc(d, axis, s0, ns, true, st); });
  phase(h, K_GEMM_FINAL_U, [&](int s0, int ns) {
    dd::launch_gemm(d, axis, s0, ns, d.K2, false, sdNT, d.N, dd::DIM_T, dd::DIM_RNEW, d.oBu, d.T, d.U, true,
                    (int64_t)d.N * d.R, nullptr, false, -1, true, false, st);
  });
  phase(h, K_GEMM_FINAL_V, [&](int s0, int ns) {
    dd::launch_gemm(d, axis, s0, ns, d.AL2, false, sdMT, d.M, dd::DIM_T, dd::DIM_RNEW, d.oBv, d.T, d.V, true,
                    (int64_t)d.M * d.R, d.isw, false, -1, false, false, st, /*set_rank=*/true);
  });
}

void enqueue_collision(dd_dlra_handle h) {
  const Dev& d = h->d;
  hipStream_t st = h->stream;
  const int64_t sdMT = (int64_t)d.M * d.T, sdNT = (int64_t)d.N * d.T;
  phase(h, K_COLL_PREP, [&](int s0, int ns) { dd::launch_coll_prep(d, s0, ns, st); });
  phase(h, K_COLL_KSTEP, [&](int s0, int ns) { dd::launch_coll_kstep(d, s0, ns, st); });
  // QR of K1; the last product writes U^1 = Q / h straight into the state
  chol_qr3(h, 0, dd::DIM_R, d.K1, d.K2, sdNT, d.N, true, d.U, (int64_t)d.N * d.R, nullptr, 1.0 / d.h, K_GEMM_QR_KC,
           K_GEMM_QR_KC_IP);
  phase(h, K_COLL_REDUCE, [&](int s0, int ns) { dd::launch_coll_reduce(d, s0, ns, st); });
  phase(h, K_COLL_SSTEP, [&](int s0, int ns) { dd::launch_coll_sstep(d, s0, ns, st); });
  phase(h, K_COLL_LSTEP, [&](int s0, int ns) { dd::launch_coll_lstep(d, s0, ns, st); });
  // weighted QR of L1 (Algorithm 3, step 5): V^1 = Q / sqrt(w) straight into
  // the state, S^1 = RL^T from the last Cholesky pass
  chol_qr3(h, 0, dd::DIM_R, d.AL, d.AL2, sdMT, d.M, false, d.V, (int64_t)d.M * d.R, d.isw, 1.0, K_GEMM_QR_LC,
           K_GEMM_QR_LC_IP, d.S);
}


// ---------------------------------------------------------------- wide plan

dd::XSrc xsrc(const void* p, int64_t sd, int ld, int dim, bool is64, int side = 0, bool rowscale = false,
              int face = 0) {
  dd::XSrc x;
  x.p = p;
  x.sd = sd;
  x.ld = ld;
  x.dim = dim;
  x.side = side;
  x.rowscale = rowscale ? 1 : 0;
  x.is64 = is64 ? 1 : 0;
  x.vec = 0;
  x.face = face;
  return x;
}

dd::XJob xjob(const dd::XSrc& x, const dd::XSrc& y, int capx, int capy, int wmode, bool sym, int out_off,
              int out_ld, double scale = 1.0, bool shift = false) {
  dd::XJob j;
  j.x = x;
  j.y = y;
  j.wmode = wmode;
  j.shift = shift ? 1 : 0;
  j.sym = sym ? 1 : 0;
  j.out_off = out_off;
  j.out_ld = out_ld;
  j.scale = scale;
  j.pa = (capx + 63) / 64;
  j.pb = (capy + 63) / 64;
  j.zbase = 0;
  j.rows_cells = 0;
  return j;
}

// partial Grams X^T X of a working array (ld rows), live ld
// Gram of X into the partial sums; wide: read by a wide kernel (d.xpN /
// d.xpM partials), else by a narrow one (d.nwgN / d.nwgM)
void w_gram(dd_dlra_handle h, int kind, int axis, const void* X, bool is64, int64_t sd, int rows, int ndim, int cap,
            bool cells, bool wide, int skip_off = -1, int np_set = 0) {
  const Dev& d = h->d;
  dd::XJobs jobs;
  jobs.n = 1;
  jobs.skip_off = skip_off;
  const dd::XSrc x = xsrc(X, sd, rows, ndim, is64);
  jobs.j[0] = xjob(x, x, cap, cap, 0, true, 0, -1);
  const int np = np_set > 0 ? np_set : (wide ? (cells ? d.xpN : d.xpM) : (cells ? d.nwgN : d.nwgM));
  phase(h, kind, [&](int s0, int ns) { dd::launch_w_xgram(d, axis, s0, ns, jobs, cells, np, h->stream); });
}

// passes of Cholesky QR of X (rows x n, n = dim ndim <= 128) for the wide
// plan, out of place, alternating between X and Y; acc: accumulate the R
// factors in the small workspace; near0: the first pass may take the
// near-identity factor too (an input orthonormal in exact arithmetic).  The
// last pass is skipped, per subdomain, after a next-to-last one that took
// the near-identity factor (its product then copies).  Returns the buffer
// holding Q.
void* w_chol_qr(dd_dlra_handle h, int axis, int ndim, void* X, void* Y, int64_t sd, int rows, bool cells, int passes,
                bool acc, int gram_kind, int gemm_kind, bool near0 = false) {
  const Dev& d = h->d;
  const int ngp = cells ? d.xpN : d.xpM;
  const int cap = ndim == dd::DIM_T ? d.T : d.R;
  void* cur = X;
  void* oth = Y;
  for (int pass = 0; pass < passes; ++pass) {
    const int skip_mode = passes < 2 ? 0 : (pass == passes - 2 ? 1 : (pass == passes - 1 ? 2 : 0));
    const int skip_off = skip_mode == 2 ? d.oSkip : -1;
    w_gram(h, gram_kind, axis, cur, false, sd, rows, ndim, cap, cells, true, skip_off);
    phase(h, K_W_CHOL, [&](int s0, int ns) {
      dd::launch_w_chol(d, axis, s0, ns, ndim, rows, ngp, acc ? (pass == 0 ? 1 : 2) : 0, 1.0, d.oRinv, d.oRacc, d.T,
                        pass > 0 || near0, h->stream, skip_mode);
    });
    phase(h, gemm_kind, [&](int s0, int ns) {
      dd::launch_w_gemm(d, axis, s0, ns, cur, false, sd, rows, ndim, ndim, d.oRinv, d.T, oth, false, sd, nullptr,
                        d.oFill, cells, true, h->stream, false, skip_off);
    });
    std::swap(cur, oth);
  }
  return cur;
}

void enqueue_advection_wide(dd_dlra_handle h, int axis, int upto = 0) {
  const Dev& d = h->d;
  hipStream_t st = h->stream;
  const int64_t sdMA = (int64_t)d.M * d.MA, sdMT = (int64_t)d.M * d.T, sdNT = (int64_t)d.N * d.T;
  const int64_t sdMR = (int64_t)d.M * d.R, sdNR = (int64_t)d.N * d.R;
  const int R = d.R, T = d.T;
  // Algorithm 4: A = sqrt(w) L0, its Gram, the SVD through the pivoted
  // Cholesky factor, V-hat = A B Sigma^-2, two Cholesky-QR passes
  phase(h, K_AUG_FORM, [&](int s0, int ns) { dd::launch_w_aug_form(d, axis, s0, ns, st); });
  // the augmentation SVD sums the Gram's partials in its one workgroup: at
  // most 8 of them
  w_gram(h, K_W_GRAM_A, axis, d.A, true, sdMA, d.M, dd::DIM_M0, d.MA, false, true, -1, d.xgM);
  phase(h, K_AUG_SVD, [&](int s0, int ns) { dd::launch_w_aug_svd(d, axis, s0, ns, st); });
  phase(h, K_GEMM_VHAT, [&](int s0, int ns) {
    dd::launch_w_gemm(d, axis, s0, ns, d.A, true, sdMA, d.M, dd::DIM_M0, dd::DIM_T, d.oCoef, d.MA, d.Qh, false, sdMT,
                      nullptr, d.oFill, false, true, st);
  });
  void* q = w_chol_qr(h, axis, dd::DIM_T, d.Qh, d.Z, sdMT, d.M, false, 2, false, K_W_GRAM_VHAT, K_GEMM_QR_VHAT, true);
  (void)q;  // two passes: V-hat is back in Qh
  if (upto == DD_PROBE_VHAT) return;
  // angular Galerkin matrices (partial layout of the narrow plan)
  {
    dd::XJobs jobs;
    const dd::XSrc qh = xsrc(d.Qh, sdMT, d.M, dd::DIM_T, false);
    jobs.n = 6;
    jobs.j[0] = xjob(xsrc(d.V, sdMR, d.M, dd::DIM_R, true, 0, true), qh, R, T, 0, false, 0, R);
    jobs.j[1] = xjob(qh, qh, T, T, 1, true, R * T, -1);
    jobs.j[2] = xjob(qh, qh, T, T, 2, true, R * T + T * T, -1);
    jobs.j[3] = xjob(qh, qh, T, T, 3, true, R * T + 2 * T * T, -1);
    jobs.j[4] = xjob(xsrc(d.V, sdMR, d.M, dd::DIM_R, true, -1, true), qh, R, T, 2, false, R * T + 3 * T * T, R);
    jobs.j[5] = xjob(xsrc(d.V, sdMR, d.M, dd::DIM_R, true, +1, true), qh, R, T, 3, false, 2 * R * T + 3 * T * T, R);
    phase(h, K_W_ANG, [&](int s0, int ns) { dd::launch_w_xgram(d, axis, s0, ns, jobs, false, d.xgM, st); });
  }
  phase(h, K_ADV_PREP, [&](int s0, int ns) { dd::launch_w_adv_prep(d, axis, s0, ns, st); });
  // Algorithm 1/2 steps 1-2: K-step, QR (three passes: K1 -> K2 -> K1 -> K2)
  if (d.rk4) {
    // K0 = U Am and the frozen ghost rows, then the four nested stages
    // K0 -> K2 -> K1 -> K2 -> K1 (each out = K0 + alpha g(in))
    phase(h, K_W_RK_PREP, [&](int s0, int ns) { dd::launch_w_rk_prep(d, axis, s0, ns, st); });
    phase(h, K_GEMM_K0, [&](int s0, int ns) {
      dd::launch_w_gemm(d, axis, s0, ns, d.U, true, sdNR, d.N, dd::DIM_R, dd::DIM_T, d.oAm, d.R, d.K3, true, sdNT,
                        nullptr, -1, true, true, st);
    });
    const void* ins[4] = {d.K3, d.K2, d.K1, d.K2};
    void* outs[4] = {d.K2, d.K1, d.K2, d.K1};
    for (int stg = 0; stg < 4; ++stg) {
      const double alpha = d.dt / (double)(4 - stg);
      phase(h, K_W_RK_KSTEP, [&](int s0, int ns) {
        dd::launch_w_rk_kstep(d, axis, s0, ns, alpha, ins[stg], outs[stg], st);
      });
    }
  } else {
    phase(h, K_KSTEP, [&](int s0, int ns) { dd::launch_w_kstep(d, axis, s0, ns, st); });
  }
  if (upto == DD_PROBE_K1) return;
  void* Q = w_chol_qr(h, axis, dd::DIM_T, d.K1, d.K2, sdNT, d.N, true, 3, true, K_W_GRAM_K, K_GEMM_QR_K);
  if (upto == DD_PROBE_U1) return;
  // step 3: spatial Galerkin matrix and the face products, S-step
  {
    dd::XJobs jobs;
    const dd::XSrc qa = xsrc(Q, sdNT, d.N, dd::DIM_T, false);
    const dd::XSrc ql = xsrc(Q, sdNT, d.N, dd::DIM_T, false, 0, false, 1);
    const dd::XSrc qhf = xsrc(Q, sdNT, d.N, dd::DIM_T, false, 0, false, 2);
    jobs.n = 5;
    jobs.j[0] = xjob(qa, qa, T, T, 0, false, 0, -1, 1.0, true);
    const int oX = 2 * T * T;
    jobs.j[1] = xjob(ql, xsrc(d.U, sdNR, d.N, dd::DIM_R, true, 0, false, 1), T, R, 0, false, oX, T);
    jobs.j[2] = xjob(qhf, xsrc(d.U, sdNR, d.N, dd::DIM_R, true, 0, false, 2), T, R, 0, false, oX + T * R, T);
    jobs.j[3] = xjob(ql, xsrc(d.U, sdNR, d.N, dd::DIM_R, true, -1, false, 2), T, R, 0, false, oX + 2 * T * R, T);
    jobs.j[4] = xjob(qhf, xsrc(d.U, sdNR, d.N, dd::DIM_R, true, +1, false, 1), T, R, 0, false, oX + 3 * T * R, T);
    phase(h, K_W_SPATIAL, [&](int s0, int ns) { dd::launch_w_xgram(d, axis, s0, ns, jobs, true, d.xgN, st); });
  }
  phase(h, K_ADV_SSTEP, [&](int s0, int ns) { dd::launch_w_adv_sstep(d, axis, s0, ns, st); });
  if (upto == DD_PROBE_S2) return;
  // steps 4-5: L-step, weighted QR (AL -> AL2 -> AL -> AL2)
  phase(h, K_LSTEP, [&](int s0, int ns) { dd::launch_w_lstep(d, axis, s0, ns, st); });
  if (upto == DD_PROBE_L1) return;
  void* QL = w_chol_qr(h, axis, dd::DIM_T, d.AL, d.AL2, sdMT, d.M, false, 3, true, K_W_GRAM_L, K_GEMM_QR_L);
  // Algorithm 5: truncation, then rotate the bases into the state
  phase(h, K_TRUNC, [&](int s0, int ns) { dd::launch_w_trunc(d, axis, s0, ns, st); });
  phase(h, K_GEMM_FINAL_U, [&](int s0, int ns) {
    dd::launch_w_gemm(d, axis, s0, ns, Q, false, sdNT, d.N, dd::DIM_T, dd::DIM_RNEW, d.oBu, d.T, d.U, true, sdNR,
                      nullptr, -1, true, false, st);
  });
  phase(h, K_GEMM_FINAL_V, [&](int s0, int ns) {
    dd::launch_w_gemm(d, axis, s0, ns, QL, false, sdMT, d.M, dd::DIM_T, dd::DIM_RNEW, d.oBv, d.T, d.V, true, sdMR,
                      d.isw, -1, false, false, st, /*set_rank=*/true);
  });
}

void enqueue_collision_wide(dd_dlra_handle h) {
  const Dev& d = h->d;
  hipStream_t st = h->stream;
  const int64_t sdMT = (int64_t)d.M * d.T, sdNT = (int64_t)d.N * d.T, sdNR = (int64_t)d.N * d.R;
  const int R = d.R;
  phase(h, K_COLL_PREP, [&](int s0, int ns) { dd::launch_w_coll_prep(d, s0, ns, st); });
  phase(h, K_COLL_KSTEP, [&](int s0, int ns) { dd::launch_w_coll_kstep(d, s0, ns, st); });
  w_gram(h, K_W_GRAM_KC, 0, d.K1, false, sdNT, d.N, dd::DIM_R, R, true, false);  // read by the narrow Cholesky QR
  // QR of K1 (stored ranks <= 64: the narrow Cholesky-QR kernels); the last
  // product writes U^1 = Q / h into the state
  chol_qr3(h, 0, dd::DIM_R, d.K1, d.K2, sdNT, d.N, true, d.U, (int64_t)d.N * d.R, nullptr, 1.0 / d.h, K_GEMM_QR_KC,
           K_GEMM_QR_KC_IP);
  {
    dd::XJobs jobs;
    const dd::XSrc u = xsrc(d.U, sdNR, d.N, dd::DIM_R, true);
    dd::XSrc qv = xsrc(d.Qsrc, d.N, d.N, dd::DIM_R, true);
    qv.vec = 1;
    const double h2 = d.h * d.h;
    jobs.n = 3;
    jobs.j[0] = xjob(u, u, R, R, 4, true, 0, R, h2);
    jobs.j[1] = xjob(u, u, R, R, 5, true, R * R, R, h2);
    jobs.j[2] = xjob(u, qv, R, 1, 0, false, 2 * R * R, R, h2);
    phase(h, K_W_COLL_REDUCE, [&](int s0, int ns) { dd::launch_w_xgram(d, 0, s0, ns, jobs, true, d.nwgN, st); });
  }
  phase(h, K_COLL_SSTEP, [&](int s0, int ns) { dd::launch_coll_sstep(d, s0, ns, st); });
  phase(h, K_COLL_LSTEP, [&](int s0, int ns) { dd::launch_coll_lstep(d, s0, ns, st); });
  chol_qr3(h, 0, dd::DIM_R, d.AL, d.AL2, sdMT, d.M, false, d.V, (int64_t)d.M * d.R, d.isw, 1.0, K_GEMM_QR_LC,
           K_GEMM_QR_LC_IP, d.S);
}

void enqueue_step(dd_dlra_handle h) {
  if (h->d.wide) {
    enqueue_advection_wide(h, 0);
    enqueue_advection_wide(h, 1);
    enqueue_collision_wide(h);
    return;
  }
  enqueue_advection(h, 0);
  enqueue_advection(h, 1);
  enqueue_collision(h);
}

dd_status check_flags(dd_dlra_handle h) {
  unsigned flags = 0;
  HIPCHK(hipMemcpy(&flags, h->d.flags, sizeof(unsigned), hipMemcpyDeviceToHost));
  if (flags & (dd::FLAG_NONFINITE | dd::FLAG_JACOBI_NOCONV)) {
    h->err = "device reported:";
    if (flags & dd::FLAG_NONFINITE) h->err += " non-finite factors;";
    if (flags & dd::FLAG_JACOBI_NOCONV) h->err += " Jacobi did not converge;";
    return DD_ENUMERIC;
  }
  if (flags & dd::FLAG_RANK_CLAMP) {
    h->err = "a rank rule exceeded its capacity (strict_caps)";
    return DD_ERANK;
  }
  return DD_OK;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================

extern "C" {

dd_status dd_dlra_workspace_size(const dd_dlra_config* cfg, size_t* bytes) {
  std::string e = validate(cfg);
  if (!e.empty()) {
    g_err = e;
    return DD_EINVAL;
  }
  if (!bytes) {
    g_err = "bytes is NULL";
    return DD_EINVAL;
  }
  *bytes = make_layout(cfg).bytes;
  return DD_OK;
}

dd_status dd_dlra_create(const dd_dlra_config* cfg, const int32_t* rank0, const double* const* U0,
                         const double* const* S0, const double* const* V0, void* d_workspace, size_t ws_bytes,
                         void* hip_stream, dd_dlra_handle* out) {
  if (!out) {
    g_err = "out is NULL";
    return DD_EINVAL;
  }
  *out = nullptr;
  std::string e = validate(cfg);
  if (!e.empty()) {
    g_err = e;
    return DD_EINVAL;
  }
  Layout L = make_layout(cfg);
  e = check_factors(cfg, L, rank0, U0, S0, V0);
  if (!e.empty()) {
    g_err = e;
    return DD_EINVAL;
  }
  if (d_workspace && ws_bytes < L.bytes) {
    g_err = "workspace too small: need " + std::to_string(L.bytes) + " bytes";
    return DD_EINVAL;
  }
  static bool kernels_ready = false;
  if (!kernels_ready) {
    dd::init_kernels();
    dd::init_wide_kernels();
    kernels_ready = true;
  }
  hipError_t serr = hipSuccess;
  double* sptr = scratch_on_current_device(&serr);
  if (!sptr) {
    g_err = std::string("hipGetSymbolAddress of the static scratch failed: ") + hipGetErrorString(serr);
    return DD_EHIP;
  }
  dd_dlra_handle h = new dd_dlra_s();
  h->cfg = *cfg;
  h->noalloc_scratch = sptr;
  h->cfg.omega_x = h->cfg.omega_y = h->cfg.w = nullptr;
  h->cfg.sigma_s = h->cfg.sigma_a = h->cfg.Q = nullptr;
  auto fail = [&](dd_status st) {
    g_err = h->err;
    dd_dlra_destroy(h);
    return st;
  };
  if (hip_stream) {
    h->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
      h->err = "hipStreamCreate failed";
      return fail(DD_EHIP);
    }
    h->own_stream = true;
  }
  if (d_workspace) {
    h->ws = d_workspace;
    h->ws_bytes = ws_bytes;
  } else {
    if (hipMalloc(&h->ws, L.bytes) != hipSuccess) {
      h->ws = nullptr;
      h->err = "hipMalloc of " + std::to_string(L.bytes) + " bytes failed";
      return fail(DD_ENOMEM);
    }
    h->own_ws = true;
    h->ws_bytes = L.bytes;
  }
  fill_dev(h->d, L, cfg, (char*)h->ws);
  Dev& d = h->d;
  {
    // one round of resident workgroups covers the batch: each wavefront then
    // walks many strips with its loads running ahead of its products
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0) {
      h->err = "cannot query the compute-unit count";
      return fail(DD_EHIP);
    }
    // the wide plan's workgroups of low-rank subdomains exit at once (column
    // chunks beyond their ranks), so it takes more of them per subdomain:
    // the high-rank subdomains then spread over more compute units
    const int occ = d.wide ? 4 : dd::ts_resident_wgs(d);
    const int per_sd = std::max(1, ncu * occ / d.nsub);
    d.nwgN = std::min(per_sd, L.nwgN);
    d.nwgM = std::min(per_sd, L.nwgM);
    set_wide_partials(d);
  }
  if (hipMemsetAsync(h->ws, 0, L.bytes, h->stream) != hipSuccess) {
    h->err = "hipMemsetAsync failed";
    return fail(DD_EHIP);
  }
  // directions
  {
    std::vector<double> in(5 * (size_t)d.M);
    for (int q = 0; q < d.M; ++q) {
      in[q] = cfg->omega_x[q];
      in[d.M + q] = cfg->omega_y[q];
      in[2 * d.M + q] = cfg->w[q];
      in[3 * d.M + q] = sqrt(cfg->w[q]);
      in[4 * d.M + q] = 1.0 / sqrt(cfg->w[q]);
    }
    if (hipMemcpyAsync(d.omx, in.data(), in.size() * 8, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess) {
      h->err = "upload of directions failed";
      return fail(DD_EHIP);
    }
  }
  // fields in subdomain-local order
  {
    std::vector<double> cs((size_t)d.nsub * d.N), ct(cs.size()), qq(cs.size());
    for (int s = 0; s < d.nsub; ++s) {
      const int sx = s % d.px, sy = s / d.px;
      for (int iy = 0; iy < d.lny; ++iy)
        for (int ix = 0; ix < d.lnx; ++ix) {
          const size_t g = (size_t)(sy * d.lny + iy) * cfg->nx + sx * d.lnx + ix;
          const size_t l = (size_t)s * d.N + iy * d.lnx + ix;
          cs[l] = cfg->sigma_s[g];
          ct[l] = cfg->sigma_s[g] + cfg->sigma_a[g];
          qq[l] = cfg->Q[g];
        }
    }
    if (hipMemcpyAsync(d.cs, cs.data(), cs.size() * 8, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(d.ct, ct.data(), ct.size() * 8, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(d.Qsrc, qq.data(), qq.size() * 8, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess) {
      h->err = "upload of fields failed";
      return fail(DD_EHIP);
    }
  }
  dd_status st = upload_factors(h, rank0, U0, S0, V0);
  if (st != DD_OK) return fail(st);
  st = upload_inflow_layers(h, cfg);
  if (st != DD_OK) return fail(st);
  *out = h;
  return DD_OK;
}

dd_status dd_dlra_step(dd_dlra_handle h, int32_t n_steps) {
  if (!h) return DD_EINVAL;
  if (n_steps < 0) {
    h->err = "n_steps must be >= 0";
    return DD_EINVAL;
  }
  if (h->cfg.exec_mode == DD_EXEC_BATCHED_GRAPH) {
    if (!h->gexec) {
      HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
      h->capturing = true;
      enqueue_step(h);
      h->capturing = false;
      hipError_t ce = hipStreamEndCapture(h->stream, &h->graph);
      if (ce != hipSuccess) {
        h->err = std::string("hipStreamEndCapture: ") + hipGetErrorString(ce);
        return DD_EHIP;
      }
      HIPCHK(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
    }
    for (int i = 0; i < n_steps; ++i) HIPCHK(hipGraphLaunch(h->gexec, h->stream));
  } else {
    for (int i = 0; i < n_steps; ++i) enqueue_step(h);
  }
  HIPCHK(hipGetLastError());
  return DD_OK;
}

namespace {

void drop_graph(dd_dlra_handle h) {
  if (h->gexec) {
    (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
  }
  if (h->graph) {
    (void)hipGraphDestroy(h->graph);
    h->graph = nullptr;
  }
}

}  // namespace

dd_status dd_dlra_set_tiling(dd_dlra_handle h, int32_t wg_per_subdomain) {
  if (!h) return DD_EINVAL;
  if (wg_per_subdomain < 1) {
    h->err = "wg_per_subdomain must be >= 1";
    return DD_EINVAL;
  }
  Dev& d = h->d;
  HIPCHK(hipStreamSynchronize(h->stream));
  const int capN = std::max(1, (int)(d.gpStride / d.gpTile));
  const int w = std::min((int)wg_per_subdomain, capN);
  d.nwgN = std::min(w, d.ntN);
  d.nwgM = std::min(w, d.ntM);
  set_wide_partials(d);
  drop_graph(h);
  return DD_OK;
}

dd_status dd_dlra_autotune(dd_dlra_handle h, int32_t steps, int32_t* wg_per_subdomain, double* ms_per_step) {
  if (!h) return DD_EINVAL;
  if (steps < 1) {
    h->err = "steps must be >= 1";
    return DD_EINVAL;
  }
  if (h->profiling) {
    h->err = "autotune while kernel profiling is on";
    return DD_ESTATE;
  }
  Dev& d = h->d;
  HIPCHK(hipStreamSynchronize(h->stream));
  // the trials run real steps: the whole workspace (state, ranks, flags,
  // scratch) is kept aside and put back after each trial
  void* snap = nullptr;
  if (hipMalloc(&snap, h->ws_bytes) != hipSuccess) {
    h->err = "hipMalloc of the autotune snapshot failed";
    return DD_ENOMEM;
  }
  auto restore = [&]() { return hipMemcpyAsync(h->ws, snap, h->ws_bytes, hipMemcpyDeviceToDevice, h->stream); };
  hipError_t e = hipMemcpyAsync(snap, h->ws, h->ws_bytes, hipMemcpyDeviceToDevice, h->stream);
  int dev = 0, ncu = 0;
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const int capN = std::max(1, (int)(d.gpStride / d.gpTile));
  const int base = std::max(1, ncu * dd::ts_resident_wgs(d) / d.nsub);
  std::vector<int> cands;
  for (int c : {base / 4, base / 2, base, 2 * base, 4 * base, 8 * base, 16 * base}) {
    const int v = std::max(1, std::min(c, capN));
    if (std::find(cands.begin(), cands.end(), v) == cands.end()) cands.push_back(v);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const int ntN = d.ntN, ntM = d.ntM;
  int best = -1;
  float best_ms = 0.0f;
  for (size_t i = 0; i < cands.size() && e == hipSuccess; ++i) {
    d.nwgN = std::min(cands[i], ntN);
    d.nwgM = std::min(cands[i], ntM);
    set_wide_partials(d);
    drop_graph(h);
    dd_status st = dd_dlra_step(h, 1);  // warm-up (captures the graph in graph mode)
    if (st != DD_OK) {
      e = hipErrorUnknown;
      break;
    }
    e = hipEventRecord(e0, h->stream);
    if (e == hipSuccess && dd_dlra_step(h, steps) != DD_OK) e = hipErrorUnknown;
    if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess) e = restore();
    if (e == hipSuccess && (best < 0 || ms < best_ms)) {
      best = cands[i];
      best_ms = ms;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  (void)hipFree(snap);
  drop_graph(h);
  if (e != hipSuccess || best < 0) {
    h->err = "autotune trial failed";
    return DD_EHIP;
  }
  d.nwgN = std::min(best, ntN);
  d.nwgM = std::min(best, ntM);
  set_wide_partials(d);
  if (wg_per_subdomain) *wg_per_subdomain = best;
  if (ms_per_step) *ms_per_step = best_ms / steps;
  return DD_OK;
}

dd_status dd_dlra_stage(dd_dlra_handle h, int32_t stage) {
  if (!h) return DD_EINVAL;
  if (stage < 0 || stage > 2) {
    h->err = "stage must be 0, 1 or 2";
    return DD_EINVAL;
  }
  if (h->d.wide) {
    if (stage < 2) enqueue_advection_wide(h, stage);
    else enqueue_collision_wide(h);
  } else {
    if (stage < 2) enqueue_advection(h, stage);
    else enqueue_collision(h);
  }
  HIPCHK(hipGetLastError());
  return DD_OK;
}

dd_status dd_dlra_probe(dd_dlra_handle h, int32_t stage, int32_t upto, int32_t sd, int64_t cap, double* buf,
                        int32_t* rows, int32_t* cols) {
  if (!h) return DD_EINVAL;
  const Dev& d = h->d;
  if (stage < 0 || stage > 1 || upto < DD_PROBE_VHAT || upto > DD_PROBE_L1 || sd < 0 || sd >= d.nsub || !buf ||
      !rows || !cols) {
    h->err = "dd_dlra_probe: stage 0 or 1, a DD_PROBE_* phase, a subdomain index and non-NULL outputs";
    return DD_EINVAL;
  }
  if (h->d.wide) enqueue_advection_wide(h, stage, upto);
  else enqueue_advection(h, stage, upto);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(h->stream));
  int t = 0;
  HIPCHK(hipMemcpy(&t, d.tdim + sd, sizeof(int), hipMemcpyDeviceToHost));
  const bool f64 = d.prec == DD_PREC_FP64;
  const void* src = nullptr;
  int nr = 0, nc = t, ld = 0;
  bool work = true;  // an array of the working type
  switch (upto) {
    case DD_PROBE_VHAT: src = (const char*)d.Qh + (size_t)sd * d.M * d.T * (f64 ? 8 : 4); nr = d.M; ld = d.M; break;
    case DD_PROBE_K1: src = (const char*)d.K1 + (size_t)sd * d.N * d.T * (f64 ? 8 : 4); nr = d.N; ld = d.N; break;
    case DD_PROBE_U1: src = (const char*)d.K2 + (size_t)sd * d.N * d.T * (f64 ? 8 : 4); nr = d.N; ld = d.N; break;
    case DD_PROBE_L1: src = (const char*)d.AL + (size_t)sd * d.M * d.T * (f64 ? 8 : 4); nr = d.M; ld = d.M; break;
    default: src = d.small + (size_t)sd * d.smallStride + d.oP0; nr = t; ld = d.T; work = false; break;
  }
  *rows = nr;
  *cols = nc;
  if (cap < (int64_t)nr * nc) {
    h->err = "dd_dlra_probe: buffer too small";
    return DD_EINVAL;
  }
  const size_t es = (work && !f64) ? 4 : 8;
  std::vector<char> tmp((size_t)ld * nc * es);
  if (!tmp.empty()) HIPCHK(hipMemcpy(tmp.data(), src, tmp.size(), hipMemcpyDeviceToHost));
  for (int j = 0; j < nc; ++j)
    for (int i = 0; i < nr; ++i) {
      const size_t o = i + (size_t)j * ld;
      const double v = es == 8 ? ((const double*)tmp.data())[o] : (double)((const float*)tmp.data())[o];
      if (upto == DD_PROBE_S2) buf[j + (size_t)i * nr] = v;  // the slot holds S2^T
      else buf[i + (size_t)j * nr] = v;
    }
  return check_flags(h);
}

dd_status dd_dlra_profile(dd_dlra_handle h, int32_t enable) {
  if (!h) return DD_EINVAL;
  if (enable < 0) {
    h->err = "enable must be >= 0";
    return DD_EINVAL;
  }
  h->profiling = enable != 0;
  h->prof_repeat = enable > 1 ? enable : 1;
  return DD_OK;
}

dd_status dd_dlra_kernel_stats(dd_dlra_handle h, int32_t n, int64_t* launches, double* total_ms, int32_t* n_kernels) {
  if (!h) return DD_EINVAL;
  HIPCHK(hipStreamSynchronize(h->stream));
  if (h->k_ms.empty()) {
    h->k_ms.assign(K_COUNT, 0.0);
    h->k_launch.assign(K_COUNT, 0);
  }
  for (size_t i = 0; i < h->pending.size(); ++i) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, h->ev_pool[2 * i], h->ev_pool[2 * i + 1]));
    // a repeated phase counts once: its time and launches per repetition
    const auto& pd = h->pending[i];
    h->k_ms[pd.kind] += ms / pd.reps;
    h->k_launch[pd.kind] += pd.launches / pd.reps;
  }
  h->pending.clear();
  h->ev_used = 0;
  for (auto& pg : h->prof_graphs) {
    (void)hipGraphExecDestroy(pg.second);
    (void)hipGraphDestroy(pg.first);
  }
  h->prof_graphs.clear();
  if (n_kernels) *n_kernels = K_COUNT;
  for (int k = 0; k < n && k < K_COUNT; ++k) {
    if (launches) launches[k] = h->k_launch[k];
    if (total_ms) total_ms[k] = h->k_ms[k];
  }
  return DD_OK;
}

const char* dd_dlra_kernel_name(int32_t k) {
  if (k < 0 || k >= K_COUNT) return nullptr;
  return kKindName[k];
}

dd_status dd_dlra_sync(dd_dlra_handle h) {
  if (!h) return DD_EINVAL;
  HIPCHK(hipStreamSynchronize(h->stream));
  return check_flags(h);
}

dd_status dd_dlra_get_ranks(dd_dlra_handle h, int32_t* r, int32_t* t_max, int64_t* clamp_events) {
  if (!h) return DD_EINVAL;
  HIPCHK(hipStreamSynchronize(h->stream));
  const int ns = h->d.nsub;
  std::vector<int> buf(ns);
  if (r) {
    HIPCHK(hipMemcpy(buf.data(), h->d.rank, ns * sizeof(int), hipMemcpyDeviceToHost));
    for (int s = 0; s < ns; ++s) r[s] = buf[s];
  }
  if (t_max) {
    HIPCHK(hipMemcpy(buf.data(), h->d.tmax, ns * sizeof(int), hipMemcpyDeviceToHost));
    for (int s = 0; s < ns; ++s) t_max[s] = buf[s];
  }
  if (clamp_events) {
    unsigned long long c = 0;
    HIPCHK(hipMemcpy(&c, h->d.clamps, sizeof(c), hipMemcpyDeviceToHost));
    *clamp_events = (int64_t)c;
  }
  return check_flags(h);
}

dd_status dd_dlra_get_factors(dd_dlra_handle h, int32_t sd, int32_t cap, int32_t* r, double* U, double* S, double* V) {
  if (!h) return DD_EINVAL;
  const Dev& d = h->d;
  if (sd < 0 || sd >= d.nsub || !r) {
    h->err = "bad subdomain index or NULL r";
    return DD_EINVAL;
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  int rr = 0;
  HIPCHK(hipMemcpy(&rr, d.rank + sd, sizeof(int), hipMemcpyDeviceToHost));
  *r = rr;
  if (cap < rr) {
    h->err = "cap smaller than the rank";
    return DD_EINVAL;
  }
  if (U) HIPCHK(hipMemcpy(U, d.U + (size_t)sd * d.N * d.R, (size_t)d.N * rr * 8, hipMemcpyDeviceToHost));
  if (V) HIPCHK(hipMemcpy(V, d.V + (size_t)sd * d.M * d.R, (size_t)d.M * rr * 8, hipMemcpyDeviceToHost));
  if (S) {
    std::vector<double> buf((size_t)d.R * d.R);
    HIPCHK(hipMemcpy(buf.data(), d.S + (size_t)sd * d.R * d.R, buf.size() * 8, hipMemcpyDeviceToHost));
    for (int j = 0; j < rr; ++j)
      for (int i = 0; i < rr; ++i) S[i + (size_t)j * rr] = buf[i + (size_t)j * d.R];
  }
  return check_flags(h);
}

dd_status dd_dlra_moments(dd_dlra_handle h, double* rho, double* jx, double* jy, int32_t dst_is_device) {
  if (!h) return DD_EINVAL;
  if (!rho) {
    h->err = "rho is NULL";
    return DD_EINVAL;
  }
  if ((jx == nullptr) != (jy == nullptr)) {
    h->err = "jx and jy must both be given or both be NULL";
    return DD_EINVAL;
  }
  const Dev& d = h->d;
  const int nmom = jx ? 3 : 1;
  dd::launch_moments(d, nmom, h->stream);
  const size_t n = (size_t)h->cfg.nx * h->cfg.ny;
  double* dst[3] = {rho, jx, jy};
  const hipMemcpyKind kind = dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  for (int m = 0; m < nmom; ++m) HIPCHK(hipMemcpyAsync(dst[m], d.rho + m * n, n * 8, kind, h->stream));
  if (dst_is_device) return DD_OK;
  HIPCHK(hipStreamSynchronize(h->stream));
  return check_flags(h);
}

dd_status dd_dlra_moments_noalloc(dd_dlra_handle h, double* rho, double* jx, double* jy) {
  if (!h) return DD_EINVAL;
  if (!rho) {
    h->err = "rho is NULL";
    return DD_EINVAL;
  }
  if ((jx == nullptr) != (jy == nullptr)) {
    h->err = "jx and jy must both be given or both be NULL";
    return DD_EINVAL;
  }
  const Dev& d = h->d;
  if (d.nsub > NOALLOC_MAX_SUB) {
    h->err = "dd_dlra_moments_noalloc: " + std::to_string(d.nsub) + " subdomains need more than the " +
             std::to_string(NOALLOC_DOUBLES * sizeof(double)) + "-byte static scratch (at most " +
             std::to_string(NOALLOC_MAX_SUB) + " subdomains)";
    return DD_EINVAL;
  }
  dd::launch_moments_twopass(d, jx ? 3 : 1, h->noalloc_scratch, rho, jx, jy, h->stream);
  HIPCHK(hipGetLastError());
  return DD_OK;
}

dd_status dd_dlra_set_factors(dd_dlra_handle h, const int32_t* rank, const double* const* U, const double* const* S,
                              const double* const* V) {
  if (!h) return DD_EINVAL;
  dd_dlra_config c = h->cfg;
  Layout L;
  L.R = h->d.R;
  L.N = h->d.N;
  L.M = h->d.M;
  L.nsub = h->d.nsub;
  // orthonormality check needs the weights: read them back from the device
  std::vector<double> w(h->d.M);
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipMemcpy(w.data(), h->d.w, w.size() * 8, hipMemcpyDeviceToHost));
  c.w = w.data();
  std::string e = check_factors(&c, L, rank, U, S, V);
  if (!e.empty()) {
    h->err = e;
    return DD_EINVAL;
  }
  return upload_factors(h, rank, U, S, V);
}

dd_status dd_dlra_force_ranks(dd_dlra_handle h, const int32_t* t, const int32_t* r_out) {
  if (!h) return DD_EINVAL;
  const int ns = h->d.nsub;
  std::vector<int> f(4 * ns, -1);
  for (int i = 0; i < 2 * ns; ++i) {
    if (t) f[i] = t[i];
    if (r_out) f[2 * ns + i] = r_out[i];
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipMemcpy(h->d.force, f.data(), f.size() * sizeof(int), hipMemcpyHostToDevice));
  h->d.forced = (t || r_out) ? 1 : 0;
  drop_graph(h);  // a captured graph holds the old kernel arguments
  return DD_OK;
}

dd_status dd_dlra_destroy(dd_dlra_handle h) {
  if (!h) return DD_OK;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  for (auto& pg : h->prof_graphs) {
    (void)hipGraphExecDestroy(pg.second);
    (void)hipGraphDestroy(pg.first);
  }
  if (h->own_ws && h->ws) (void)hipFree(h->ws);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return DD_OK;
}

const char* dd_dlra_last_error(dd_dlra_handle h) {
  if (!h) return g_err.c_str();
  return h->err.c_str();
}

}  // extern "C"
