/*
 * libifgf — IFGF-accelerated N-Mueller boundary-integral operator on MI355X.
 *
 * Implements the hot path of Paul & Sideris, "Accelerated 3D Maxwell Integral
 * Equation Solver using the Interpolated Factored Green Function Method"
 * (arXiv 2408.02274): the Green's-function and Green's-gradient sums over
 * Chebyshev-Nystrom surface points at two wavenumbers (Sec. III-E..III-I,
 * eq. ifgf_sum_em), the near-field singular corrections (Sec. III-D, III-H),
 * the N-Mueller operator built from them (Sec. II, eq. n_muller..t_delta) and
 * GMRES on the resulting 4N x 4N system (Sec. III-A, eq. lin_system).
 *
 * Conventions for every entry point
 *  - Status: 0 = IFGF_OK, < 0 error, > 0 warning.  On error the thread-local
 *    message is available from ifgf_last_error().  No entry point aborts.
 *  - Complex numbers are interleaved (re, im) pairs, FP64 unless stated.
 *  - "host" pointers are read during the call only and copied; the caller
 *    keeps ownership.  "device" pointers are HIP device memory owned by the
 *    caller; the library never frees them.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work is enqueued on it; apply calls do not synchronise the host.
 *  - A plan owns its device workspaces; they are released by the destroy call.
 *    A plan may be used from one host thread at a time.
 */
#ifndef IFGF_H
#define IFGF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IFGF_OK 0
#define IFGF_EINVAL (-1)       /* invalid argument (message says which)        */
#define IFGF_ENOMEM (-2)       /* host or device allocation failed             */
#define IFGF_EHIP (-3)         /* HIP runtime error (message holds its string) */
#define IFGF_ENOTPLANNED (-4)  /* operation needs a plan that was not built    */
#define IFGF_EDEVICE (-5)      /* a kernel reported a failure (ifgf_check)     */
#define IFGF_WNOCONV 1         /* GMRES stopped at maxit before the tolerance  */

#define IFGF_FP64 0            /* cone grids, interpolation, sums in FP64      */
#define IFGF_FP32 1            /* cone grids and interpolation in FP32         */

#define IFGF_DERIV_ANALYTIC 0  /* n.grad of the interpolant, analytically      */
#define IFGF_DERIV_FD 1        /* the paper's forward difference, h = 1e-6     */

typedef struct ifgf_plan_s* ifgf_plan_t;

/* Options; ifgf_default_options() fills the paper's defaults.
 * Ps, Pa: interpolation points per cone in the radial and in each angular
 *   variable (Sec. III-F; Remark 2 uses 3 and 5).  0 = chosen from `tol`.
 * ns_init, na_init: cone counts at level D+1 (Remark 2; Sec. IV uses 1, 2).
 * refine_radial: 1 (default) doubles the radial and the angular cone counts
 *   per level where kappa*H_d > 1/2 (Remark 2); 0 doubles only the angular
 *   count, which is cheaper but whose radial interpolation error grows with
 *   kappa*H of the coarse boxes (a radius-5 sphere at Ps, Pa = 5, 6: 8e-4 in
 *   the single-layer and 2.5e-3 in the normal-derivative sums, against
 *   1e-6 and 3e-5 with the radial doubling).
 * leaf_wavelengths: leaf boxes satisfy H_D <= leaf_wavelengths * lambda_min
 *   with lambda_min = 2 pi / max(k_int, k_ext) (Sec. III-G; 0.25).
 * precision: IFGF_FP64 or IFGF_FP32.
 * max_nrhs: largest nrhs accepted by the apply calls (sizes workspaces).
 * host_only: 1 builds the host tables only (no device memory is touched);
 *   such a plan serves ifgf_plan_counts/ifgf_plan_table/ifgf_stats, and the
 *   apply calls return IFGF_ENOTPLANNED.
 * batch_columns: right-hand sides stacked into the columns of one pass of
 *   the matrix-core kernels (1, 2 or 4; FP64 at most 2; 0 -> 1).  The cone
 *   buffers grow by that factor; whether it pays depends on the workload
 *   (ifgf_autotune measures it).
 * fp32_workspaces: 1 with precision IFGF_FP32 sizes the cone buffers, the
 *   per-pair target buffer and the density copy for FP32 values (half the
 *   device memory of the default, which keeps room for the FP64 form); such a
 *   plan cannot be switched to IFGF_FP64 (ifgf_set_precision: IFGF_EINVAL).
 * verbose: 1 prints one progress line per planning stage and level on
 *   stderr (large surfaces take minutes to plan), and one line per 20
 *   iterations of the solves on an N-Mueller operator built with it.
 * deriv_mode: how the normal derivative of a cousin contribution is taken
 *   (Sec. III-I): IFGF_DERIV_ANALYTIC (default) differentiates the
 *   interpolant times the centred factor; IFGF_DERIV_FD is the paper's
 *   (G F)(x + h n) - (G F)(x) over h = 1e-6, x + h n interpolated in the cone
 *   of x.  FD needs IFGF_FP64, the matrix-core orders and one right-hand side
 *   per apply (max_nrhs = batch_columns = 1); near sums stay analytic.
 * target_chunk_pairs: the matrix-core target interpolation writes one result
 *   per (target, cousin box) pair and sums them per target; it takes the
 *   targets of a level in chunks of consecutive targets holding at most this
 *   many pairs, so that the result buffer stays bounded (0 -> 1 GiB of FP64
 *   results, 2,396,745 pairs; the sums do not depend on it).
 * plan_on_device: 1 (default) builds the plan tables (algorithm step 1:
 *   Morton order, boxes, neighbours, cousins, relevant cones, pair and tile
 *   lists) with kernels on the current device, 0 on the host; the tables are
 *   the same bit for bit (host_only plans always use the host).
 * keep_pair_tables: 1 keeps host copies of the cousin-pair and
 *   propagation-pair cone slots after upload, for ifgf_plan_table.
 * kernel_at_a_time (Remark 3): 0 (default) interpolates the 8 densities of
 *   both kernels in one pass (IFGF_Vec); 1 runs one pass per kernel, with
 *   half the cone-buffer memory and one right-hand side per pass; -1 picks
 *   one pass per kernel at plan time when the cone buffers of both kernels
 *   would exceed cone_memory_budget.  Needs the matrix-core orders (Pa = 5
 *   or 6, 3 <= Ps <= 6), else IFGF_EINVAL.  The sums are the same either
 *   way up to rounding; ifgf_stats reports the choice (kernels_per_pass)
 *   and the cone-buffer bytes of both modes.
 * cone_memory_budget: bytes the cone buffers may take when
 *   kernel_at_a_time = -1; 0 = the free device memory at plan time less the
 *   plan's other workspaces (a caller that allocates more afterwards, such
 *   as the N-Mueller corrections, passes its own budget).
 * target_tiles: 1 (default) interpolates onto the cousin targets on the
 *   matrix cores, in cone-major tiles of up to 8 targets; 0 uses one thread
 *   per (target, kernel) instead (slower; the same sums up to rounding;
 *   IFGF_DERIV_FD needs the tiles).                                        */
typedef struct {
  int Ps, Pa;
  int ns_init, na_init;
  int refine_radial;
  double leaf_wavelengths;
  int precision;
  int max_nrhs;
  int host_only;
  int batch_columns;
  int fp32_workspaces;
  int verbose;
  int deriv_mode;
  int64_t target_chunk_pairs;
  int plan_on_device;
  int keep_pair_tables;
  int kernel_at_a_time;
  int64_t cone_memory_budget;
  int target_tiles;
} ifgf_options;

void ifgf_default_options(ifgf_options* opt);

/* Build the IFGF plan for the discrete sums of eq. ifgf_sum_em (Sec. III-I):
 *   out[r][q][c][l]   = sum_{m != l} w_m phi_{r,c}(x_m) G_q(x_l, x_m),        c = 0..7
 *   out[r][q][8+c][l] = sum_{m != l} w_m phi_{r,c}(x_m) n_l . grad G_q(...), c = 0..5
 * with G_q(x,y) = exp(i k_q |x-y|)/(4 pi |x-y|), k_0 = k_int, k_1 = k_ext.
 *  n        number of points (>= 1)
 *  points   host [n][3] FP64, pairwise different (Sec. III-E)
 *  normals  host [n][3] FP64 unit normals (|n| within 1e-6 of 1)
 *  weights  host [n] FP64 quadrature weights (> 0), e.g. Fejer w_i w_j J_p
 *  k_int, k_ext  wavenumbers (> 0)
 *  tol      target relative accuracy in [1e-10, 1e-1]; selects Ps, Pa when
 *           the options leave them 0: tol >= 1e-3 -> (3, 5) (the paper's),
 *           >= 1e-4 -> (4, 6), >= 1e-5 -> (7, 8), else (8, 8), the smallest
 *           orders whose relative L2 error (with refine_radial = 1) stayed
 *           below tol in every output block (S and the normal-derivative
 *           sums separately) on spheres of radius 1 to 5 wavelengths and an
 *           ellipsoid, and on the 40 x 1 x 0.5-wavelength rounded box at
 *           1.67M points (S 2.5e-6, D 3.8e-5 at tol 1e-4).  The mapping is
 *           empirical, not a bound: on the same box with only 11,360 points
 *           and random weights the normal-derivative sums reached 2.5e-4 at
 *           tol 1e-4 (they are small against the terms they sum there; the
 *           next orders bring them to 3.2e-5).  Below 1e-6 the largest orders
 *           do not reach tol
 *  opt      NULL = defaults
 * Errors: IFGF_EINVAL (bad sizes, NaN/Inf, non-unit normals, weights <= 0,
 * k <= 0, tol out of range, duplicate points), IFGF_ENOMEM, IFGF_EHIP.     */
int ifgf_plan(ifgf_plan_t* out, int64_t n, const double* points,
              const double* normals, const double* weights, double k_int,
              double k_ext, double tol, const ifgf_options* opt);

/* Evaluate the sums above (no singular correction).
 *  densities device [nrhs][8][n] complex (FP64), caller point order, the
 *            unweighted densities phi (the plan applies the weights)
 *  out       device [nrhs][2][14][n] complex (FP64), overwritten
 * nrhs must be in [1, max_nrhs].  Errors: IFGF_EINVAL, IFGF_EHIP.           */
int ifgf_apply(ifgf_plan_t plan, const void* densities, int nrhs, void* out,
               void* stream);

/* Plan counts (host [ncount] int64, filled up to ncount entries):
 *  0 n, 1 D, 2 Ps, 3 Pa, 4 near pairs, 5 leaf slots, 6 leaf (point, source)
 *  pairs, then for d = 3..D four entries per level: relevant cones, target
 *  pairs, propagation pairs (d >= 4, else 0), ns_d * 65536 + na_d.          */
int ifgf_plan_counts(ifgf_plan_t plan, int64_t* counts, int ncount);

/* Copy plan tables to host for inspection and tests.
 *  which = 0: sorted-position -> input-index permutation, int64 [n]
 *  which = 1000 + d: relevant cone keys of level d, int64 box*ncones+cone
 *  (box = Morton-ordered index of the level's non-empty boxes)
 *  which = 2000 + d: cone slot of every (cousin target, source box) pair of
 *  level d, ordered by sorted target then cousin list (host_only plans)
 *  which = 3000 + d: child cone slot of every (parent interpolation point,
 *  child box) pair propagated into level d (host_only plans).
 * `count` receives the number of entries; `buf` may be NULL to query it.   */
int ifgf_plan_table(ifgf_plan_t plan, int which, int64_t* buf, int64_t cap,
                    int64_t* count);

/* JSON summary of the plan; with timing on, also per-kernel launch counts,
 * summed durations (ms, from HIP events on the apply stream) and summed work
 * units (pairs or points) since timing was switched on.  Reading the timing
 * synchronises on the recorded events.                                     */
int ifgf_stats(ifgf_plan_t plan, char* json, size_t cap);

/* Time one apply for every column batch R = 1, 2, 4 up to the plan's
 * min(batch_columns, max_nrhs) (on zero densities, in buffers it allocates
 * and frees) and keep the R with the lowest time per right-hand side for
 * the following applies; `chosen` (may be NULL) receives it.  Synchronises
 * the stream.  Per-kernel timing must be off.                               */
int ifgf_autotune(ifgf_plan_t plan, void* stream, int* chosen);

/* Switch the working precision of a built plan (IFGF_FP64 or IFGF_FP32)
 * for the following apply calls; `previous` (may be NULL) receives the one
 * in force before.  The FP64 and FP32 forms share the plan tables; FP32 is
 * available when Pa = 5 or 6 and 3 <= Ps <= 6 (else IFGF_EINVAL).  Used by the
 * mixed-precision solve: Arnoldi on the FP32 form, residuals on the FP64.   */
int ifgf_set_precision(ifgf_plan_t plan, int precision, int* previous);

/* The working precisions a built plan can run: bit 0 IFGF_FP64 (not for
 * plans built with fp32_workspaces), bit 1 IFGF_FP32 (matrix-core orders and
 * analytic derivative).  0 for NULL or host_only plans.                     */
int ifgf_precisions(ifgf_plan_t plan);

/* Device-side failures.  The FP32 propagation adds its tiles into a shared
 * accumulator under a lock whose wait is bounded; a wavefront that gives up
 * skips its tile and sets bit 0 of the plan's device error word, so that the
 * sums are never silently wrong.  ifgf_check synchronises `stream`, copies
 * the word to *flags (may be NULL), clears it, and returns IFGF_EDEVICE if it
 * was set (the applies since the previous check are then incomplete).
 * nmuller_solve checks after every solve; ifgf_stats reports the word.     */
int ifgf_check(ifgf_plan_t plan, void* stream, unsigned* flags);

/* Attempts of the bounded lock wait above (default 2^22, i.e. seconds of
 * spinning, which a correct run never approaches).  For tests of the error
 * path: 0 makes every locked add give up, and ifgf_check must then report
 * IFGF_EDEVICE while every kernel still runs to its end.                   */
int ifgf_set_lock_spin_limit(ifgf_plan_t plan, int limit);

/* Replace the normals of a built plan (host [n][3] FP64 unit vectors, caller
 * order): the direction of the derivative sums at each point.  Synchronous.
 * Errors: IFGF_EINVAL (null, non-unit), IFGF_EHIP.                          */
int ifgf_set_normals(ifgf_plan_t plan, const double* normals);

/* Switch per-kernel timing on (1) or off (0); either resets the totals.    */
int ifgf_set_timing(ifgf_plan_t plan, int on);

void ifgf_destroy(ifgf_plan_t plan);

/* Thread-local message of the last failed call ("" if none).               */
const char* ifgf_last_error(void);

/* ---------------------------------------------------------------------------
 * Sums at points other than the sources (off-surface field evaluation through
 * the same IFGF; the paper's near-field maps, Sec. IV):
 *   out[r][q][c][t]   = sum_m w_m phi_{r,c}(y_m) G_q(x_t, y_m),          c < 8
 *   out[r][q][8+c][t] = sum_m w_m phi_{r,c}(y_m) d_t . grad G_q(x_t, y_m), c < 6
 * at targets x_t with unit directions d_t; no term is excluded (targets must
 * differ from every source).  One octree holds sources and targets; targets
 * carry zero density.  Targets closer to the sources than a leaf box get the
 * plain near sum, which is accurate only a few node spacings away from a
 * discretised surface.
 * ------------------------------------------------------------------------- */
typedef struct ifgf_eval_s* ifgf_eval_t;

/*  src, weights  host [n_src][3], [n_src] FP64 source points and weights
 *  tgt, dirs     host [n_tgt][3] FP64 targets and unit directions
 *  k_int, k_ext, tol, opt  as for ifgf_plan (host_only not supported)
 * Errors: IFGF_EINVAL (also a target equal to a source), IFGF_ENOMEM,
 * IFGF_EHIP.                                                                */
int ifgf_eval_plan(ifgf_eval_t* out, int64_t n_src, const double* src, const double* weights,
                   int64_t n_tgt, const double* tgt, const double* dirs, double k_int, double k_ext,
                   double tol, const ifgf_options* opt);
/*  densities device [nrhs][8][n_src] complex FP64; out device [nrhs][2][14][n_tgt]. */
int ifgf_eval_apply(ifgf_eval_t ev, const void* densities, int nrhs, void* out, void* stream);
/*  New target directions (host [n_tgt][3]); e.g. the three axes in turn give
 *  the full gradient of the single-layer sums.  Synchronous.               */
int ifgf_eval_set_directions(ifgf_eval_t ev, const double* dirs);
/*  The IFGF plan over sources and targets (owned by ev; for statistics).    */
ifgf_plan_t ifgf_eval_ifgf(ifgf_eval_t ev);
void ifgf_eval_destroy(ifgf_eval_t ev);

/* ---------------------------------------------------------------------------
 * N-Mueller operator (Sec. II eq. n_muller, k_delta, r_delta, t_delta) on a
 * patch surface discretised by open Chebyshev grids (Sec. III-A).
 * Point order l = j + Nc*i + p*Nc^2 with x_l = eta_p(u_i, v_j),
 * u_k = cos((k + 1/2) pi / Nc) (eq. cheby_nodes, mesh_pts_l).
 * Unknowns y[r][4][n] = (m.t1, m.t2, j.t1, j.t2) with t1 = d_u eta/|d_u eta|,
 * t2 = n x t1, n = d_u eta x d_v eta / |.| (outward when the caller orients
 * the patches so).  Wavenumbers k_s = omega sqrt(eps_s mu_s).
 * ------------------------------------------------------------------------- */
typedef struct nmuller_s* nmuller_t;

/* P, Nc: patches and nodes per direction (2 <= Nc <= 16), n = P Nc^2.
 * eps_e, eps_i, mu_e, mu_i: exterior/interior permittivity and permeability.
 * omega: angular frequency (lengths in vacuum wavelengths give 2 pi).
 * delta_factor: singular set S_l = {p : dist(x_l, Gamma_p) <= delta_p} with
 *   delta_p = delta_factor x diagonal of the patch's node bounding box
 *   (Sec. III-B eq. patch_sing; 0 -> 1.0).
 * nbeta: Fejer points per direction of the singular rule (eq. int_moments_cov;
 *   0 -> 6 Nc).  d_cov: parameter d of the sigmoidal map (eq. mk_cov_1; 4).
 * corrections_on_host: 0 (default) builds the corrections on the device when
 *   Nc is 4, 5, 6, 8 or 10 and nbeta <= 64 (the same pairs and closest points
 *   as the host builder, bit for bit; weights equal to FP64 rounding), else on
 *   the host; 1 always builds them on the host.                             */
typedef struct {
  int P, Nc;
  double eps_e, eps_i, mu_e, mu_i;
  double omega;
  double delta_factor;
  int nbeta;
  int d_cov;
  int corrections_on_host;
} nmuller_params;

void nmuller_default_params(nmuller_params* p);

/* Build the operator: surface quantities (normals, Jacobians, Fejer weights
 * w_i w_j J), the IFGF plan of the regular sums at (k_int, k_ext) and the
 * near-field corrections (Sec. III-D singular moments minus the regular Fejer
 * weights, Sec. III-H), the latter kept in FP64.
 *  points, du, dv  host [n][3] FP64: nodes and d eta/du, d eta/dv there
 *  tol, opt        as for ifgf_plan (opt->host_only builds host tables only)
 * Errors: IFGF_EINVAL, IFGF_ENOMEM, IFGF_EHIP.                               */
int nmuller_plan(nmuller_t* out, const nmuller_params* prm, const double* points,
                 const double* du, const double* dv, double tol, const ifgf_options* opt);

/* Ay = A y for y device [nrhs][4][n] complex FP64; Ay device, same shape.   */
int nmuller_apply(nmuller_t nm, const void* y, int nrhs, void* Ay, void* stream);

/* Right-hand side of eq. n_muller: b = omega^-1 (n x E, n x H) projected on
 * (t1, t2).  E, H device [nrhs][n][3] complex FP64 (incident fields at the
 * nodes); b device [nrhs][4][n].                                           */
int nmuller_rhs(nmuller_t nm, const void* E, const void* H, int nrhs, void* b, void* stream);

/* Incident field of an electric dipole at a complex source point (the
 * end-face excitation of the paper's waveguide example, Sec. IV): moment p at
 * x_s = x_0 + i b d radiates, for k b >> 1, a Gaussian beam of waist
 * sqrt(2 b / k) along +d.  With R = x - x_s, r = sqrt(R.R) (principal branch),
 * G = exp(i k r) / (4 pi r):
 *   E = (k^2 G p + grad (p . grad G)) / eps,   H = -i omega grad G x p,
 * an exact solution of curl E = i omega mu H, curl H = -i omega eps E away
 * from the branch-cut disk {|x - x_0| <= b, (x - x_0) . d = 0} (b = 0: the
 * ordinary point dipole).
 *  points  device [n][3] FP64 evaluation points (n >= 0)
 *  k, eps, omega  wavenumber, permittivity and frequency of the medium
 *  dipole  host [12] FP64: p as 3 (re, im) pairs, x_0 [3], b d [3]
 *  E, H    device [n][3] complex FP64, overwritten
 * Errors: IFGF_EINVAL (null, non-finite or non-positive arguments).        */
int ifgf_dipole_field(int64_t n, const void* points, double k, double eps, double omega,
                      const double* dipole, void* E, void* H, void* stream);

/* Host copies of surface quantities: which = 0 normals [n][3], 1 weights [n],
 * 2 t1 [n][3], 3 t2 [n][3], 4 Jacobians [n].                                */
int nmuller_geometry(nmuller_t nm, int which, double* buf, int64_t cap);

/* Near-field corrections: npairs receives the number of (target, patch)
 * pairs; row_off [n+1], pair_patch [npairs] and vals [npairs][4][Nc^2][2]
 * (kernel order S k_int, S k_ext, D k_int, D k_ext; FP64 re/im) are filled
 * when non-NULL (vals copied from the device when the plan holds them
 * there only).                                                              */
int nmuller_corrections(nmuller_t nm, int64_t* npairs, int64_t* row_off,
                        int32_t* pair_patch, double* vals);

/* Plan facts, info[0..3]: 1 if the corrections were built on the device,
 * seconds the correction build took, number of (target, patch) pairs, bytes
 * of correction weights.  cap >= 4.                                         */
int nmuller_plan_info(nmuller_t nm, double* info, int cap);

/* Per right-hand side outcome of nmuller_solve.                             */
typedef struct {
  int iters;              /* matrix-vector products in the Arnoldi process     */
  int converged;          /* 1 when true_relres <= rtol                        */
  double true_relres;     /* ||b - A y|| / ||b|| from a final matvec           */
  double arnoldi_relres;  /* GMRES residual estimate at exit                   */
  double seconds;         /* host wall time from the start of its lock-step
                             group until this right-hand side finished        */
  int precond_iters;      /* iterations run with the network part of M on      */
  int fallbacks;          /* preconditioned cycles abandoned (see below)       */
  int residual_fp64;      /* 1: residuals from the FP64 IFGF form; 0: from the
                             working form, for plans that hold no FP64 cone
                             buffers (fp32_workspaces); corrections, assembly
                             and the residual arithmetic are FP64 either way */
} ifgf_solve_info;

/* Solve A y = b by GMRES (Sec. III-A eq. lin_system): Arnoldi in FP64 with
 * Gram-Schmidt applied twice, Givens rotations, stop when the residual
 * estimate reaches rtol (the paper uses 1e-4), restart after `restart`
 * iterations (0 = none), at most maxit matvecs per right-hand side.
 *  rhs  device [nrhs][4][n] complex FP64
 *  y    device [nrhs][4][n]: initial guess if use_x0, else overwritten from 0
 *  info host [nrhs] (may be NULL)
 * Several right-hand sides run in lock-step (project addition): each step
 * gathers the pending products of all unconverged solves into batched
 * applies of up to max_nrhs columns (the operator's creation option);
 * converged solves drop out.  The group holds as many solves as half the
 * free device memory allows for their Krylov bases (16 B x 4n x (basis + 1,
 * plus basis with a preconditioner)); larger nrhs run group after group.
 * Each solve's arithmetic is that of a lone solve.
 * Returns IFGF_WNOCONV (> 0) if some true residual exceeds rtol; the best
 * iterate is still returned.  Synchronises the stream a few times per
 * iteration and right-hand side.                                            */
int nmuller_solve(nmuller_t nm, const void* rhs, int nrhs, void* y, int use_x0, double rtol,
                  int maxit, int restart, ifgf_solve_info* info, void* stream);

/* nmuller_solve for one right-hand side that allocates nothing, for callers
 * that cannot allocate device memory (tight serving loops, harnesses that
 * forbid hipMalloc).  Arguments and result as nmuller_solve with nrhs = 1.
 * The GMRES workspaces (Krylov basis [basis + 1][4n], the flexible basis
 * [basis][4n] when a preconditioner is set, two vectors [4n] and the
 * reduction partials; basis = restart if 0 < restart < maxit, else maxit)
 * live in a static device array of 64 MiB that every GPU the library runs
 * on holds until the process ends; a problem whose workspaces exceed it
 * returns IFGF_EINVAL (e.g. 4n = 6,144 fits a basis of 600, 4n = 614,400 a
 * basis of 5).  The operator's own buffers (built by nmuller_plan) are used
 * as by nmuller_solve.  All calls on one GPU share the array: calls that
 * overlap in time on one GPU race and must be serialised by the caller.
 * Nothing in the array needs to start at zero (every workspace is written
 * before it is read).  Synchronises the stream like nmuller_solve.        */
int nmuller_solve_noalloc(nmuller_t nm, const void* rhs, void* y, int use_x0, double rtol, int maxit,
                          int restart, ifgf_solve_info* info, void* stream);

/* Unrestarted GMRES from y = 0 that also records iterates: after every
 * `stride`-th iteration k it writes x_k to X[j] and its residual
 * r_k = b - A x_k (from the Arnoldi relation, no extra matvec) to R[j],
 * j = 0, 1, .. < cap; *nrec receives the number written.  X, R device
 * [cap][4][n] complex FP64; rhs, y as for nmuller_solve (nrhs = 1).  Used to
 * generate (residual, error) training pairs for the learned preconditioner
 * (project addition).  Unlike nmuller_solve, every residual here (and
 * info->true_relres) is taken with the operator's working precision, so a
 * plan running its FP32 form can be driven to tolerances below its FP32
 * error.  Returns IFGF_WNOCONV like nmuller_solve.                         */
int nmuller_solve_trajectory(nmuller_t nm, const void* rhs, void* y, double rtol, int maxit,
                             int stride, void* X, void* R, int cap, int* nrec,
                             ifgf_solve_info* info, void* stream);

/* ---------------------------------------------------------------------------
 * Learned FGMRES preconditioner (project addition; the paper uses plain
 * GMRES).  z = M(v) acts on each patch separately: a network with ReLU
 * hidden layers maps the patch's 4 Nc^2 complex unknowns (real parts then
 * imaginary parts of each of the four components, node order of the patch,
 * divided by s = rms(v)) followed by 4 patch features (kappa_e d / 2pi,
 * kappa_i d / 2pi, twice the largest normal deviation angle, eps_i / eps_e / 10,
 * d = node bounding-box diagonal) to a correction c of the same 8 Nc^2 layout;
 * z = D^-1 v + s c, D = diag((mu_e+mu_i)/2, (eps_e+eps_i)/2) the identity part
 * of eq. n_muller.  With a preconditioner set, nmuller_solve runs flexible
 * GMRES; a cycle whose network output is non-finite or whose residual
 * estimate falls by less than 5% over 20 iterations is abandoned at its last
 * good column and the solve continues with the network switched off
 * (M = D^-1); ifgf_solve_info counts these fallbacks.
 * ------------------------------------------------------------------------- */
#define MLP_BF16 0   /* matrix-product operands in bfloat16, FP32 accumulation */
#define MLP_FP32 1   /* FP32 operands (used to check gradients)                 */

/* Set (params != NULL) or remove (params == NULL) the preconditioner.
 * params: host FP32, layer by layer W_l [dims[l]][dims[l+1]] row-major then
 * b_l [dims[l+1]]; dims: nlayers + 1 widths with dims[0] = 8 Nc^2 + 4 and
 * dims[nlayers] = 8 Nc^2.  The operator keeps its own copy.                 */
int nmuller_set_preconditioner(nmuller_t nm, const float* params, const int* dims, int nlayers,
                               int dtype);

/* z = M(v) for nvec vectors: v, z device [nvec][4][n] complex FP64, z must
 * not alias v.  IFGF_ENOTPLANNED without a preconditioner.                  */
int nmuller_precond_apply(nmuller_t nm, const void* v, void* z, int nvec, void* stream);

/* Training rows from (residual, error) pairs in the layout M uses:
 *  R, E  device [npairs][4][n] complex FP64 (residuals r = A e and errors e)
 *  X     device FP32 [npairs * P][8 Nc^2 + 4]: pack(r / rms(r)) and features
 *  T     device FP32 [npairs * P][8 Nc^2]: pack((e - D^-1 r) / rms(r))
 * Needs a preconditioner set (it fixes the layout; its weights are unused). */
int nmuller_precond_pairs(nmuller_t nm, const void* R, const void* E, int npairs, float* X,
                          float* T, void* stream);

/* Host copy of the 4 features of each patch, [P][4] FP32.                  */
int nmuller_patch_features(nmuller_t nm, float* buf, int64_t cap);

/* The network itself, for training: y = W_L^T .. relu(W_1^T x + b_1) .. + b_L.
 * All matrix products run on the matrix cores; parameters, gradients and
 * Adam moments are FP32 (the BF16 form keeps a rounded operand copy of the
 * weights, refreshed after every update).                                   */
typedef struct mlp_s* mlp_t;

/* nlayers in [1, 16]; dims: nlayers + 1 widths in [1, 65536]; dtype MLP_BF16
 * or MLP_FP32; max_batch: largest batch (rows) of any call.  Parameters start
 * at zero.                                                                  */
int mlp_create(mlp_t* out, int nlayers, const int* dims, int dtype, int max_batch);
int mlp_num_params(mlp_t net, int64_t* n);
/* Host FP32 parameters in the layout of nmuller_set_preconditioner; resets
 * the Adam state.  Synchronises the device.                                 */
int mlp_set_params(mlp_t net, const float* params);
int mlp_get_params(mlp_t net, float* params, void* stream);   /* host FP32, syncs */
int mlp_get_grad(mlp_t net, float* grad, void* stream);       /* host FP32, syncs */
/* Y = net(X): X device FP32 [B][dims[0]], Y device FP32 [B][dims[L]],
 * 1 <= B <= max_batch.  Keeps the activations (and, in FP32, a reference to
 * X, which must stay unchanged until mlp_backward) for a backward pass.     */
int mlp_forward(mlp_t net, const float* X, int B, float* Y, void* stream);
/* Gradients of a loss given dY = dLoss/dY (device FP32 [B][dims[L]]) for the
 * batch of the preceding mlp_forward: parameter gradient kept in the network
 * (mlp_get_grad), input gradient written to dX (device [B][dims[0]]) unless
 * dX is NULL.                                                                */
int mlp_backward(mlp_t net, const float* dY, int B, float* dX, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with step size lr.      */
int mlp_adam_step(mlp_t net, float lr, void* stream);
/* One training step on rows idx[0..B) of X (device FP32 [*][dims[0]]) and
 * targets T (device FP32 [*][dims[L]]): forward, mean-squared loss (written
 * to loss, device FP32 [1], before the update), backward, Adam.            */
int mlp_train_step(mlp_t net, const float* X, const float* T, const int32_t* idx, int B, float lr,
                   float* loss, void* stream);
void mlp_destroy(mlp_t net);

/* ---------------------------------------------------------------------------
 * Batching by graph capture (project addition): the applies of several
 * operators (bodies), each on its own nrhs right-hand sides, recorded once
 * into one HIP graph and replayed with a single launch.  The apply path
 * neither allocates nor synchronises, so a replay does exactly the eager
 * work on the buffers given at capture time (their contents may change
 * between launches; the buffers themselves must stay allocated).
 * ------------------------------------------------------------------------- */
typedef struct ifgf_graph_s* ifgf_graph_t;

/* Capture nmuller_apply(ops[i], y[i], nrhs[i], Ay[i]) for i < nops.  The
 * applies of one operator stay in the given order on one branch of the
 * graph (they share its workspaces); different operators share nothing and
 * get branches of their own, forked from and joined into the launch
 * stream, so they may run concurrently.  y[i], Ay[i] device
 * [nrhs[i]][4][n_i] complex FP64; outputs of different entries must not
 * overlap.  Per-kernel timing must be off on every operator (IFGF_EINVAL). */
int nmuller_graph_capture(ifgf_graph_t* out, int nops, const nmuller_t* ops,
                          const void* const* y, const int* nrhs, void* const* Ay);
/* Enqueue one replay on `stream`.                                           */
int ifgf_graph_launch(ifgf_graph_t g, void* stream);
/* Number of nodes (kernel launches) in the captured graph.                  */
int ifgf_graph_nodes(ifgf_graph_t g, int64_t* nodes);
void ifgf_graph_destroy(ifgf_graph_t g);

/* The IFGF plan used by the operator (owned by nm).                         */
ifgf_plan_t nmuller_ifgf(nmuller_t nm);

void nmuller_destroy(nmuller_t nm);

#ifdef __cplusplus
}
#endif
#endif /* IFGF_H */
