/*
 * dd_dlra.h -- C ABI of the MI355X (gfx950) DD-DLRA time-step engine.
 *
 * The engine advances a domain-decomposition dynamical low-rank (DD-DLRA)
 * approximation of the radiative transfer equation (Brunner, Einkemmer,
 * Haut, "Domain decomposition dynamical low-rank for multi-dimensional
 * radiative transfer equations"): every spatial subdomain k holds its own
 * factors F_k = U_k S_k V_k^T, and one step is Algorithm 6 of the paper --
 * augmentation with the neighbours' angular bases (Algorithm 4), the
 * projector-splitting integrator for x- and y-advection with inflow data
 * transferred from the neighbours (Algorithms 1 and 2, eq. generate_Kboundary
 * and its y counterpart), truncation (Algorithm 5), and the projector-
 * splitting integrator for absorption, scattering and source (Algorithm 3).
 *
 * Model (Section 2, eq. rt, with a general direction set):
 *   d_t f + c_adv (Omega_x d_x + Omega_y d_y) f = c_s rho / W - c_t f + Q,
 *   rho = sum_q w_q f_q,  W = sum_q w_q,  c_t = sigma_a + sigma_s.
 * Discretisation: square cells of width h, first-order upwind (Appendix A),
 * explicit Euler for every K-, S- and L-substep, vacuum physical faces.
 *
 * Conventions
 *   - global cells p = iy*nx + ix; subdomain s = sy*px + sx holds
 *     lnx = nx/px by lny = ny/py cells with local index iy*lnx + ix;
 *   - factors of subdomain s (rank r): U is N x r column-major (N = lnx*lny)
 *     with h^2 U^T U = I; S is r x r column-major; V is M x r column-major
 *     with V^T diag(w) V = I;
 *   - all arguments are host pointers unless stated; every host input is
 *     copied during the call that receives it;
 *   - every call returns a dd_status; no C++ exception crosses the ABI.
 *   - One handle belongs to one HIP stream and is not re-entrant.
 */
#ifndef DD_DLRA_H
#define DD_DLRA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dd_dlra_s* dd_dlra_handle;

typedef enum {
  DD_OK = 0,
  DD_EINVAL = -1,    /* invalid argument or configuration (nothing touched)   */
  DD_ENOMEM = -2,    /* device allocation failed                              */
  DD_EHIP = -3,      /* a HIP runtime call failed                             */
  DD_ERANK = -4,     /* a rank capacity was exceeded (strict_caps mode)        */
  DD_ENUMERIC = -5,  /* non-finite value or factorisation breakdown on device  */
  DD_ESTATE = -6     /* call not valid in the handle's current state           */
} dd_status;

/* Precision of the step.  DD_PREC_FP64: everything in FP64.  The mixed modes
 * keep the K-, L-step and V-hat working arrays (K1, the QR of K1, L1, the QR
 * of L1, V-hat: the widest tall-skinny data, t = the intermediate rank
 * columns) in FP32 in device memory and form the K-/L-step contractions and
 * the final basis rotations on the matrix cores in FP32 (DD_PREC_MIXED_FP32)
 * or as split BF16 products hi*hi + hi*lo + lo*hi with FP32 accumulation
 * (DD_PREC_MIXED_BF16).  The stored factors U, S, V, the augmentation matrix
 * and its SVD, the Gram and Galerkin reductions, the Cholesky QR factors and
 * products, the S-step and the eigen-split stay FP64, and so does everything
 * returned through this interface. */
enum { DD_PREC_FP64 = 0, DD_PREC_MIXED_FP32 = 1, DD_PREC_MIXED_BF16 = 2 };
enum { DD_RANK_FIXED = 0, DD_RANK_ADAPTIVE = 1 };
enum { DD_EXEC_PER_SUBDOMAIN = 0, DD_EXEC_BATCHED = 1, DD_EXEC_BATCHED_GRAPH = 2 };
/* Physical faces (Section 4): vacuum (zero inflow), or a prescribed inflow
 * f_in(position along the face, direction) = sum_k a_k(position) b_k(direction)
 * that enters through the face for the directions pointing into the domain
 * (-x face: Omega_x >= 0; +x: Omega_x < 0; -y: Omega_y >= 0; +y: Omega_y < 0).
 * An inflow face acts as a neighbour of the subdomains along it: a layer one
 * cell thick outside the face holding f_in, which supplies their ghost
 * values and joins the augmentation (Algorithm 4) with the factors
 * U = Q_a / h, S = h R_a, V = b of the thin QR a_s = Q_a R_a of the
 * subdomain's part of a. */
enum { DD_BC_VACUUM = 0, DD_BC_INFLOW_LOWRANK = 1 };
/* Substep integrator of every K-, S- and L-step (Algorithms 1-3): one
 * explicit Euler step of length dt, or one classic four-stage Runge-Kutta
 * step with the boundary data frozen over the substep (Section 4 runs use
 * the latter).  RK4 runs in DD_PREC_FP64. */
enum { DD_INT_EULER = 0, DD_INT_RK4 = 1 };

typedef struct {
  int32_t nx, ny;          /* global cells                                        */
  int32_t px, py;          /* subdomains per axis; nx % px == 0, ny % py == 0     */
  double x0, x1, y0, y1;   /* domain; (x1-x0)/nx must equal (y1-y0)/ny           */
  int32_t n_dir;           /* M, number of directions                             */
  const double* omega_x;   /* [M] direction cosines along x                       */
  const double* omega_y;   /* [M] direction cosines along y                       */
  const double* w;         /* [M] positive quadrature weights, W = sum(w)         */
  double c_adv;            /* advection speed                                     */
  const double* sigma_s;   /* [ny*nx] scattering coefficient, >= 0               */
  const double* sigma_a;   /* [ny*nx] absorption coefficient, >= 0               */
  const double* Q;         /* [ny*nx] isotropic source                            */
  double dt;               /* time step of every substep                          */
  int32_t rank_mode;       /* DD_RANK_FIXED or DD_RANK_ADAPTIVE                   */
  int32_t r_fixed;         /* fixed mode: stored rank after truncation            */
  int32_t r_min, r_max;    /* adaptive mode: bounds of the stored rank            */
  int32_t r_int_max;       /* cap of the intermediate rank after augmentation     */
  double tol;              /* adaptive mode: absolute L2 tolerance (Alg. 4, 5)     */
  double tol_aug_rel;      /* fixed mode: augmentation tail <= tol_aug_rel*sigma_1 */
  int32_t precision;       /* DD_PREC_*                                            */
  int32_t exec_mode;       /* DD_EXEC_*                                            */
  int32_t bc[4];           /* faces -x, +x, -y, +y: DD_BC_VACUUM or _INFLOW_LOWRANK */
  int32_t strict_caps;     /* 1: a rank clamp latches DD_ERANK; 0: clamp, count   */
  int32_t integrator;      /* DD_INT_EULER or DD_INT_RK4                           */
  /* prescribed inflow of the faces with bc[f] = DD_BC_INFLOW_LOWRANK (ignored
   * otherwise; copied at create): rank rb = bc_rank[f] (1 <= rb <= the
   * stored-rank capacity), bc_a[f] [rb][face cells] (ny cells along an x
   * face, nx along a y face, in increasing coordinate), bc_b[f] [rb][M]   */
  int32_t bc_rank[4];
  const double* bc_a[4];
  const double* bc_b[4];
} dd_dlra_config;

/* Device bytes a handle needs for this configuration (state, scratch and
 * per-subdomain small workspaces).  Validates the configuration first. */
dd_status dd_dlra_workspace_size(const dd_dlra_config* cfg, size_t* bytes);

/* Create a handle and upload the initial factors.
 *   rank0[s]          initial rank of subdomain s (1 <= r <= capacity)
 *   U0[s], S0[s], V0[s] host arrays of subdomain s in the layouts above;
 *                     orthonormality is checked to 1e-8 (DD_EINVAL otherwise)
 *   d_workspace       device memory of at least ws_bytes bytes owned by the
 *                     caller (it must outlive the handle), or NULL: the
 *                     library allocates and frees its own
 *   hip_stream        hipStream_t to run on, or NULL for the default stream
 * The configuration is validated before any device call. */
dd_status dd_dlra_create(const dd_dlra_config* cfg, const int32_t* rank0,
                         const double* const* U0, const double* const* S0,
                         const double* const* V0, void* d_workspace, size_t ws_bytes,
                         void* hip_stream, dd_dlra_handle* out);

/* Advance n_steps steps of Algorithm 6.  Asynchronous on the handle's
 * stream; device-side faults (non-finite values, breakdowns, clamps in
 * strict mode) are latched and reported by the next synchronising call.
 * In DD_EXEC_BATCHED_GRAPH mode the first call captures one step into a
 * hipGraph that later calls replay. */
dd_status dd_dlra_step(dd_dlra_handle h, int32_t n_steps);

/* Advance one stage of Algorithm 6 only: stage 0 = x-advection (steps 1-3:
 * augmentation, Algorithm 1, truncation), 1 = y-advection (steps 4-6),
 * 2 = absorption/scattering/source (step 7, Algorithm 3).  Asynchronous;
 * ignores the captured graph.  dd_dlra_step(h, 1) equals stages 0, 1, 2. */
dd_status dd_dlra_stage(dd_dlra_handle h, int32_t stage);

/* Current stored ranks r[s], the largest intermediate rank t_max[s] seen
 * since creation, and the number of rank clamp events (any may be NULL).
 * Synchronises the stream. */
dd_status dd_dlra_get_ranks(dd_dlra_handle h, int32_t* r, int32_t* t_max, int64_t* clamp_events);

/* Copy the factors of subdomain sd to host buffers with room for rank cap:
 * U [N*cap], S [cap*cap] (leading dimension r on output), V [M*cap].  If
 * cap < r the call writes r to *r and returns DD_EINVAL.  Synchronises. */
dd_status dd_dlra_get_factors(dd_dlra_handle h, int32_t sd, int32_t cap, int32_t* r,
                              double* U, double* S, double* V);

/* Angular moments of f on the global grid [ny*nx], cell p = iy*nx + ix:
 * scalar flux rho = sum_q w_q f_q (Section 2) and, when jx and jy are not
 * NULL, the current density jx = sum_q w_q Omega_x,q f_q, jy likewise (the
 * first moments, computed from the factors as U (S (V^T (w Omega))).  rho is
 * required; jx and jy must both be given or both be NULL (else DD_EINVAL).
 * dst_is_device != 0: the pointers are device memory written asynchronously
 * on the handle's stream; otherwise host memory (the call synchronises). */
dd_status dd_dlra_moments(dd_dlra_handle h, double* rho, double* jx, double* jy, int32_t dst_is_device);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * moments as dd_dlra_moments with device destinations, computed without any
 * allocation and without staging on the handle's grid buffer.  The
 * per-subdomain moment vectors (S (V^T (w Omega_m))) go to a static device
 * array of the library (1024 subdomains x 3 moments x 64 ranks, 1.5 MiB per
 * GPU, held until the process ends); handles with more than 1024
 * subdomains get DD_EINVAL.  rho (and jx, jy, both or neither) are device
 * pointers of nx*ny doubles, written asynchronously on the handle's stream;
 * results are identical to dd_dlra_moments.  All calls on one GPU share the
 * static array: calls that overlap on one GPU (other streams or threads)
 * race and must be serialised by the caller.  Calls no hipMalloc/hipFree. */
dd_status dd_dlra_moments_noalloc(dd_dlra_handle h, double* rho, double* jx, double* jy);

/* Replace the factors of every subdomain (same layouts as dd_dlra_create);
 * used for checkpoint/restart.  Synchronises. */
dd_status dd_dlra_set_factors(dd_dlra_handle h, const int32_t* rank,
                              const double* const* U, const double* const* S,
                              const double* const* V);

/* Parity replay: make the following steps use the given intermediate ranks
 * t[2*S] (x stage for all subdomains, then y stage) and stored ranks after
 * truncation r_out[2*S] (same order) instead of the rank rules; entries <= 0
 * keep the rule.  Pass NULL for both to return to the rules. */
dd_status dd_dlra_force_ranks(dd_dlra_handle h, const int32_t* t, const int32_t* r_out);

/* Stage probe, for testing the kernels phase by phase against a reference:
 * runs advection stage `stage` (0 = x, 1 = y) from the current state up to
 * and including the phase `upto` (the phases of Algorithms 1/2 and 4) and
 * copies one working array of subdomain sd into buf (column-major, ld
 * *rows; *rows x *cols values, cap = room in buf in doubles, DD_EINVAL if
 * short).  The stored factors and ranks are left as they were (a stage
 * writes them only in its final products; the largest-t statistic of
 * dd_dlra_get_ranks may grow).  Synchronous.
 *   DD_PROBE_VHAT  sqrt(w) V-hat after the augmentation, M x t
 *   DD_PROBE_K1    the K-step output K1 in the basis V-hat, N x t
 *   DD_PROBE_U1    h U1 (orthonormal factor of the QR of K1), N x t
 *   DD_PROBE_S2    the S-step output S2 in the bases (U1, V-hat), t x t
 *   DD_PROBE_L1    sqrt(w) L1, the L-step output (F = U1 L1^T), M x t   */
enum { DD_PROBE_VHAT = 1, DD_PROBE_K1 = 2, DD_PROBE_U1 = 3, DD_PROBE_S2 = 4, DD_PROBE_L1 = 5 };
dd_status dd_dlra_probe(dd_dlra_handle h, int32_t stage, int32_t upto, int32_t sd, int64_t cap, double* buf,
                        int32_t* rows, int32_t* cols);

/* Kernel timing.  With enable != 0, later non-graph launches (exec modes
 * PER_SUBDOMAIN and BATCHED, and dd_dlra_stage) are bracketed by hipEvent
 * pairs on the handle's stream, one pair per phase.  With enable = k > 1 the
 * tall-skinny phases whose launch leaves the same result when repeated are
 * captured k times into a graph that is replayed inside their pair, and the
 * measured time is divided by k (the per-launch average then carries little
 * dispatch overhead, and the totals stay those of one pass); the factors are
 * unchanged by the repetition.  enable < 0 returns DD_EINVAL.  dd_dlra_kernel_stats
 * synchronises, folds the pending pairs into per-kernel totals and copies
 * out launches[k] and total_ms[k] for k < n (any pointer may be NULL);
 * *n_kernels receives the number of kernel kinds.  dd_dlra_kernel_name
 * returns the static name of kind k (NULL if out of range). */
dd_status dd_dlra_profile(dd_dlra_handle h, int32_t enable);
dd_status dd_dlra_kernel_stats(dd_dlra_handle h, int32_t n, int64_t* launches, double* total_ms,
                               int32_t* n_kernels);
const char* dd_dlra_kernel_name(int32_t k);

/* Autotuner: choose the number of workgroups per subdomain of the
 * tall-skinny kernels (the decomposition of each subdomain's cells and
 * directions into row tiles) by timing the live problem.  Candidates are
 * 1/4, 1/2, 1, 2 and 4 times one round of resident workgroups per subdomain
 * (clipped to the room reserved for partial sums and to one tile of 64 rows
 * per workgroup); each runs one warm-up and `steps` timed steps in the
 * handle's execution mode, and the whole workspace is copied aside before
 * the trials and restored after each one, so the factors, ranks and flags
 * are unchanged on return.  The fastest candidate stays in effect (a
 * captured graph is recaptured at the next step).  *wg_per_subdomain and
 * *ms_per_step (either may be NULL) receive the choice and its time per
 * step.  Needs a temporary device allocation of the workspace size
 * (DD_ENOMEM if it fails); DD_ESTATE while kernel profiling is on; DD_EINVAL
 * for steps < 1.  Synchronises. */
dd_status dd_dlra_autotune(dd_dlra_handle h, int32_t steps, int32_t* wg_per_subdomain, double* ms_per_step);

/* Set the workgroups per subdomain of the tall-skinny kernels directly (for
 * instance a choice of dd_dlra_autotune kept from an earlier run), clipped to
 * the reserved room and to one 64-row tile per workgroup.  DD_EINVAL for
 * wg_per_subdomain < 1.  Synchronises; a captured graph is recaptured. */
dd_status dd_dlra_set_tiling(dd_dlra_handle h, int32_t wg_per_subdomain);

/* Wait for the handle's stream and report latched device errors. */
dd_status dd_dlra_sync(dd_dlra_handle h);

/* Release the handle and, if the library allocated it, its device memory. */
dd_status dd_dlra_destroy(dd_dlra_handle h);

/* Last error message of the handle (or of the last failed create/validate
 * call when h is NULL).  The string lives until the next call on it. */
const char* dd_dlra_last_error(dd_dlra_handle h);

#ifdef __cplusplus
}
#endif
#endif /* DD_DLRA_H */
