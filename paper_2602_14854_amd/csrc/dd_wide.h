// Definitions shared by the wide-plan kernels (dd_wide.hip) and the host
// launch plan (dd_api.hip).
#pragma once

#include "dd_internal.h"

namespace dd {

// capacities of the wide plan
constexpr int WCAP_R = 64;    // stored rank
constexpr int WCAP_T = 128;   // intermediate rank
constexpr int WCAP_A = 192;   // augmentation width (3 stored ranks)

// One operand of a row reduction (kw_xgram).
struct XSrc {
  const void* p;   // base of the array of all subdomains
  int64_t sd;      // elements per subdomain
  int ld;          // leading dimension (rows of the full array)
  int dim;         // DIM_* selector of the column count (own subdomain)
  int side;        // 0: own subdomain; -1 / +1: neighbour along the stage axis (its stored rank)
  int rowscale;    // 1: values multiplied by sqrt(w[row]) (direction rows)
  int is64;        // 1: FP64 array; 0: working-type array of the precision mode
  int vec;         // 1: a per-cell vector (one column, FP64, indexed [s][row])
  int face;        // 0: all rows; 1: the low face cells; 2: the high face cells
};

// out[i, j] = scale sum_rows w(row) X[row, i] Y'[row, j] into the partial of
// the workgroup at out_off with leading dimension out_ld (<= 0: the live
// column count of X).  wmode: 0 none, 1 Omega of the stage axis, 2
// 1[Omega >= 0], 3 1[Omega < 0], 4 c_s, 5 c_t.  shift: Y'[p] = Y[p + e] -
// Y[p] (zero beyond the high face).  sym: X = Y, blocks a <= b, mirrored.
struct XJob {
  XSrc x, y;
  int wmode, shift, sym;
  int out_off, out_ld;
  double scale;
  int pa, pb;       // 64-column blocks of X and Y by capacity
  int zbase;        // first blockIdx.z of the job (set by the launcher)
  int rows_cells;   // rows are cells (set by the launcher)
};

constexpr int XJOBS_MAX = 8;
struct XJobs {
  XJob j[XJOBS_MAX];
  int n;
  int skip_off = -1;  // >= 0: a subdomain whose small-workspace slot here is set writes nothing
};

void launch_w_gemm(const Dev& d, int axis, int sd0, int nsd, const void* X, bool x64, int64_t xsd, int rows,
                   int kdim, int ndim, int boff, int bld, void* Y, bool y64, int64_t ysd, const double* rowscale,
                   int fill_off, bool rows_are_cells, bool exact, hipStream_t st, bool set_rank = false,
                   int skip_off = -1);
void launch_w_aug_form(const Dev& d, int axis, int sd0, int nsd, hipStream_t st);
void launch_w_kstep(const Dev& d, int axis, int sd0, int nsd, hipStream_t st);
void launch_w_lstep(const Dev& d, int axis, int sd0, int nsd, hipStream_t st);
void launch_w_coll_kstep(const Dev& d, int sd0, int nsd, hipStream_t st);
void launch_w_xgram(const Dev& d, int axis, int sd0, int nsd, XJobs jobs, bool cells, int np, hipStream_t st);
// near: a Gram within 1e-3 of the identity takes the symmetric factor from
// the binomial series instead of the Cholesky factorisation
// skip_mode 1 records in the skip slot whether the pass took the
// near-identity factor (its output is then orthonormal to rounding); a pass
// with skip_mode 2 does nothing for a subdomain whose slot is set
void launch_w_chol(const Dev& d, int axis, int sd0, int nsd, int ndim, int rows, int ngp, int acc_mode,
                   double bscale, int oRinv, int oRacc, int ld, bool near, hipStream_t st, int skip_mode = 0);
void launch_w_aug_svd(const Dev& d, int axis, int sd0, int nsd, hipStream_t st);
void launch_w_adv_prep(const Dev& d, int axis, int sd0, int nsd, hipStream_t st);
void launch_w_adv_sstep(const Dev& d, int axis, int sd0, int nsd, hipStream_t st);
void launch_w_trunc(const Dev& d, int axis, int sd0, int nsd, hipStream_t st);
void launch_w_coll_prep(const Dev& d, int sd0, int nsd, hipStream_t st);
// RK4 advection K-step: frozen ghost rows, then out = K0 + alpha g(in)
void launch_w_rk_prep(const Dev& d, int axis, int sd0, int nsd, hipStream_t st);
void launch_w_rk_kstep(const Dev& d, int axis, int sd0, int nsd, double alpha, const void* in, void* out,
                       hipStream_t st);
void init_wide_kernels();

}  // namespace dd
