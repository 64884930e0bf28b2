/*
 * fftt.h -- C ABI of the MI355X (gfx950) finite-frequency traveltime
 * tomography operators.
 *
 * Method: Korta Martiartu, Boehm & Fichtner, "3D wave-equation-based
 * finite-frequency tomography for ultrasound computed tomography"
 * (arXiv:1908.03302).  The library applies the linearised cross-correlation
 * traveltime Jacobian J (the forward matrix F of eq. forward_compact) and its
 * transpose without storing it: every entry
 *
 *     J_ij = A(x_j) h(R_ij) dV,   A = -L_i / (2 pi c0^3 R_xs R_xr)
 *            (eq. Linearized_sensitivity_A),  R = R_xs + R_xr - L_i,
 *
 * is evaluated on the fly from a tabulated one-dimensional function h of the
 * detour R (the re-parameterisation of Sec. II-C, eq. Kernel_freq), truncated
 * to zero for R >= R_max, at voxel centres x_j (midpoint rule, voxel volume
 * dV).  Regularised least squares (eq. leastSquare_misfit1/_misfit) and
 * Hessian point-spread functions (eq. resolution_2) are built on top.
 *
 * Conventions shared by every call:
 *  - SI units: metres, seconds, m/s.  dc is a velocity perturbation (m/s),
 *    dT a traveltime perturbation (s).  A positive dc gives a negative dT.
 *  - Voxel (i,j,k) has its centre at origin + (i,j,k) * spacing and flat index
 *    i + nx*(j + ny*k) (x fastest).  N = nx*ny*nz.
 *  - Pair m = (source, receiver) indices into the transducer list; rows of J
 *    and entries of dT follow the caller's pair order.
 *  - Host pointers are read during the call only; the library copies what it
 *    keeps.  Device pointers (the dc / dT buffers of apply, solve and psf)
 *    are owned by the caller, must be contiguous, and must hold FP64 for
 *    FFTT_FP64 and FP32 otherwise.
 *  - Device work is enqueued on the context's stream and is asynchronous
 *    unless stated otherwise.
 *  - Every call returns a status; nothing is thrown across the ABI.  On an
 *    error nothing observable changes and fftt_last_error() describes it.
 *  - One context per host thread; calls on one context must not overlap.
 */
#ifndef FFTT_H
#define FFTT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fftt_ctx fftt_ctx;

typedef enum {
    FFTT_OK = 0,
    FFTT_E_INVALID = -1,      /* bad argument; nothing changed */
    FFTT_E_NOMEM = -2,        /* device or host allocation failed */
    FFTT_E_DEVICE = -3,       /* a HIP runtime call failed */
    FFTT_E_STATE = -4,        /* geometry or kernel table missing */
    FFTT_E_UNSUPPORTED = -5,  /* valid request outside what is built */
    FFTT_NOT_CONVERGED = 1    /* warning: result written, target not met */
} fftt_status;

typedef enum {
    FFTT_FP64 = 0,            /* FP64 evaluation, table and accumulation */
    FFTT_FP32 = 1,            /* FP32 evaluation/accumulation, FP32 table;
                                 detour formed from FP64 geometry */
    FFTT_FP32_BF16TABLE = 2   /* as FFTT_FP32 with the table held in BF16 */
} fftt_precision;

/* Create a context on HIP device `device`; work goes to `hip_stream`
 * (a hipStream_t, NULL = the legacy default stream). */
fftt_status fftt_create(fftt_ctx **out, int device, void *hip_stream);
void fftt_destroy(fftt_ctx *ctx);
/* Detail of the last error on this context; valid until the next call. */
const char *fftt_last_error(const fftt_ctx *ctx);
/* Change the stream later calls enqueue on. */
fftt_status fftt_set_stream(fftt_ctx *ctx, void *hip_stream);

/* Acquisition geometry and model grid (paper Sec. II-C: pairs x_s, x_r in a
 * water background of velocity c0; M = n_pairs rows, N = voxels columns).
 *   tx_xyz  host [n_tx][3] transducer positions; 2 <= n_tx <= 65535.
 *   pairs   host [n_pairs][2] (source, receiver), source != receiver.
 *   origin, spacing, dims: the voxel grid (spacing > 0).
 *   active_mask host [N] (0 = voxel outside the region of interest, its dc
 *           is ignored on input and written as 0 on output) or NULL (all).
 * FFTT_E_INVALID if a transducer sits on an active voxel centre. */
fftt_status fftt_set_geometry(fftt_ctx *ctx, double c0,
                              const double *tx_xyz, int64_t n_tx,
                              const int32_t *pairs, int64_t n_pairs,
                              const double origin[3], const double spacing[3],
                              const int64_t dims[3], const uint8_t *active_mask);

/* The 2D approximation (Sec. II-B, eq. forward_2D): transducers and the
 * model in (or near) one plane, the model constant along z over [z0, z1],
 * so dT = sum over pixels of (int_{z0}^{z1} K0 dz) dc(x, y) dA.  The z
 * integral is the midpoint rule on nz layers of thickness dz = (z1 - z0)/nz:
 * the operators work on the prism of nx * ny * nz voxels (layer k at z0 +
 * (k + 1/2) dz, voxel volume dA dz) with J reading dc(x, y) in every layer
 * and J^T summing the layers.  Model vectors (apply_J input, apply_JT
 * output, solves, point-spread functions, low-rank analysis) then have N =
 * nx * ny values; fftt_coverage and the Jacobi preconditioner return
 * FFTT_E_UNSUPPORTED (their absolute values and squares do not commute with
 * the layer sum); fftt_work_count counts prism evaluations.  BF16 tables
 * are not offered in this mode: apply_J, apply_JT, solve, psf,
 * hessian_apply, hessian_lowrank and autotune return FFTT_E_UNSUPPORTED for
 * FFTT_FP32_BF16TABLE (the layer sum adds Fresnel zones of alternating
 * sign, so the table's BF16 rounding is not averaged away and J^T would sit
 * at the 1e-3 bound of that precision).
 *   origin, spacing, dims: in-plane grid (pixel (0,0) centre, x fastest);
 *   active_mask: host [ny][nx] or NULL; 1 <= nz <= 4096.  Otherwise as
 *   fftt_set_geometry, which switches back to 3D. */
fftt_status fftt_set_geometry_2d(fftt_ctx *ctx, double c0, const double *tx_xyz,
                                 int64_t n_tx, const int32_t *pairs, int64_t n_pairs,
                                 const double origin[2], const double spacing[2],
                                 const int64_t dims[2], double z0, double z1, int64_t nz,
                                 const uint8_t *active_mask);

/* Kernel table of frequency band `band` (0 <= band < 4): host h[n] holds
 * h(k * r_max / (n-1)), k = 0..n-1, the function of the detour defined by
 * eq. Kernel_freq (without A).  Between nodes h is interpolated linearly;
 * for R >= r_max the kernel is zero (truncation of Sec. II-C).  All bands
 * must use the same n (2 <= n <= 16384).  With B bands set (0..B-1),
 * apply_J writes B outputs per right-hand side and apply_JT sums over bands.
 * FP32 operators: when |h[n-1]| <= 1e-6 max|h| in every band (as in the
 * tables of fftt_build_table_from_pulse), the single-precision node table
 * stores h[n-1] as 0, so h falls to 0 across the last interval below r_max
 * instead of to h[n-1]; other tables are used as given. */
fftt_status fftt_set_kernel_table(fftt_ctx *ctx, int32_t band, const double *h,
                                  int64_t n, double r_max);

/* Host helper: tabulate h from a sampled calibration pulse f(t_k), k < nt,
 * spacing dt (Sec. II-A: the source-time function measured in water), by
 * trapezoid quadrature of eq. Kernel_freq with S = |DTFT(f)|^2 and the upper
 * frequency limit read as infinity.  With r_max <= 0 the radius is chosen as
 * the smallest R beyond which |h| < 1e-7 max|h|; *r_max_out returns it.
 * h_out: host [n]. */
fftt_status fftt_build_table_from_pulse(double c0, const double *f, int64_t nt,
                                        double dt, int64_t n, double r_max,
                                        double *h_out, double *r_max_out);

/* The paper's own representation of the detour function (Sec. II-C: the
 * coefficients and arguments of the sines of eq. Kernel_freq, evaluated on
 * the fly):  h(R) = sum_{m=1}^{n} a_m sin(m beta R) for 0 <= R < r_max and 0
 * beyond.  Attaches such a series to a band whose table is already set with
 * the same r_max (re-setting the table with another r_max drops it).
 * a: host [n_terms], 1 <= n_terms <= 64; 0 < beta * r_max <= pi.  With
 * FFTT_TUNE_KERNEL_EVAL = 1 the FP32 operators (apply_J, apply_JT and the
 * solves built on them) evaluate the series instead of interpolating the
 * table; they then return FFTT_E_STATE if a band has no series and
 * FFTT_E_UNSUPPORTED where the LDS-staged kernels do not apply.  FP64,
 * BF16-table and PSF evaluations keep the table. */
fftt_status fftt_set_kernel_series(fftt_ctx *ctx, int32_t band, const double *a,
                                   int32_t n_terms, double beta, double r_max);

/* Host helper: the sine series of eq. Kernel_freq for a sampled pulse
 * (S = |DTFT(f)|^2 as above): the frequency integrals as trapezoid sums over
 * uniform nodes w_m = m dw, m = 1..n, so a_m = w_m^3 S(w_m) / sum_k w_k^2
 * S(w_k) and beta = dw / c0.  dw = 2 pi c0 / (2.5 r_max): the series is
 * periodic in R with period 2.5 r_max, so its first alias lies beyond
 * 1.5 r_max.  n is the fewest nodes reaching past the last frequency where
 * w^3 S exceeds tol times its maximum (e.g. tol = 1e-8: h within ~1e-10 of
 * max|h|, far below FP32 rounding); FFTT_E_INVALID if
 * that needs more than max_terms, or for bad arguments (r_max > 0 required).
 * a_out: host [max_terms]; *n_terms_out, *beta_out returned. */
fftt_status fftt_build_series_from_pulse(double c0, const double *f, int64_t nt,
                                         double dt, double r_max, double tol,
                                         int32_t max_terms, double *a_out,
                                         int32_t *n_terms_out, double *beta_out);

/* Build the device-side culling lists now (otherwise the first apply does).
 * Synchronises the stream. */
fftt_status fftt_prepare(fftt_ctx *ctx);

/* Work counts after prepare: pv = number of (pair, active voxel)
 * combinations of the operator with detour below the largest r_max (decided
 * in FP64, over the caller's pairs); pv_evaluated = the same over the pairs
 * the kernels evaluate (pairs with identical rows of J are evaluated once,
 * see FFTT_TUNE_RECIPROCITY); lanes = evaluation slots the kernels execute
 * per band (>= pv_evaluated, includes culling slack).  Any pointer may be
 * NULL. */
fftt_status fftt_work_count(fftt_ctx *ctx, int64_t *pv, int64_t *pv_evaluated,
                            int64_t *lanes);

/* dT = J dc (eq. forward_compact) for n_rhs right-hand sides.
 *   dc: device [n_rhs][N];  dT: device [n_rhs][B][M] (overwritten).
 * With n_rhs >= 8 and FFTT_TUNE_RHS_BATCHED = 1 (default), FP32 / BF16-table
 * operators with table evaluation, 1 to 3 bands, in 3D, the right-hand
 * sides run as batches on the matrix cores (per tile the products with
 * all of them are split-BF16 contractions, as in fftt_hessian_apply;
 * within 1e-5, norm-wise per vector, of the one-vector path; library
 * workspace: nb * (evaluated entries) floats per column, batches kept
 * under about 8 GB).  Otherwise, and for fewer right-hand sides, one
 * launch per right-hand side.  The same holds for fftt_apply_JT, whose
 * batch is the point-spread-function contraction of fftt_psf applied to
 * the data vectors (workspace nb * (kernel pairs) * ceil32(n_rhs) words). */
fftt_status fftt_apply_J(fftt_ctx *ctx, fftt_precision prec, const void *dc,
                         void *dT, int32_t n_rhs);

/* dc = J^T dT, summed over bands (the transpose used by the normal equations
 * of eq. leastSquare_misfit and the Hessian of eq. resolution_2).
 *   dT: device [n_rhs][B][M];  dc: device [n_rhs][N] (overwritten). */
fftt_status fftt_apply_JT(fftt_ctx *ctx, fftt_precision prec, const void *dT,
                          void *dc, int32_t n_rhs);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): J^T
 * exactly as fftt_apply_JT (same kernels, same results), making no
 * hipMalloc / hipFree or other allocating call.  Its work memory -- the
 * per-pair weights, B x (evaluated pairs) values of the precision's type,
 * and in the 2D mode the prism's output, nx*ny*nz values -- lives in a
 * file-scope device array of 16 MiB that every device the library runs on
 * holds until the process ends; a request that needs more returns
 * FFTT_E_INVALID.  The context must be ready: geometry and tables set and
 * prepared (fftt_prepare, or any earlier apply after the last change of
 * geometry, tables or tuning), else FFTT_E_STATE.  The array is shared by
 * every call on the device, on any context or stream, and keeps the last
 * call's contents (each call writes all it reads): calls that overlap on
 * one device race.  Not recorded by fftt_profile.
 *   dT: device [n_rhs][B][M];  dc: device [n_rhs][N] (overwritten). */
fftt_status fftt_apply_JT_noalloc(fftt_ctx *ctx, fftt_precision prec, const void *dT,
                                  void *dc, int32_t n_rhs);

/* Regularised least squares with Gaussian noise Gamma_n = sigma^2 I and
 * Gaussian prior Gamma_pr = I (eq. leastSquare_misfit1 / leastSquare_misfit):
 * minimise |J x - d|^2 / sigma^2 + alpha |x|^2 over all bands.
 *   method 0 = CGLS (conjugate gradients on the damped normal equations),
 *   method 1 = LSQR (damp = sqrt(alpha)) on the scaled system J/sigma.
 * prec FFTT_FP64: every vector and operator in FP64; otherwise operators in
 * FP32 (or BF16 table) with FP32 vectors and FP64 inner products.
 * Stops at max_iter, or once |J x - d|^2/sigma^2 <= target_misfit
 * (if > 0), or once the normal-equation residual falls by rel_tol (if > 0).
 *   d_obs: device [B][M]; x: device [N], in: x0 (used as start when
 *   opts->use_x0 != 0, else zero), out: estimate.  Synchronises once at the
 *   end (and once per iteration when a target or tolerance is set); rep
 *   receives iterations, final misfit (evaluated in the solver's
 *   arithmetic), relative normal residual and elapsed time.
 *   use_graph != 0: the second iteration is captured into a HIP graph on the
 *   context's stream and replayed for the remaining ones (one launch per
 *   iteration instead of ~20); results are identical to use_graph = 0.  The
 *   stream must not be used by other work during the solve.
 *   precond = 1 (CGLS only): Jacobi-preconditioned CG on the same normal
 *   equations, M = diag(J^T J) / sigma^2 + alpha I, the diagonal computed
 *   once per solve by fftt_coverage (FP32, staged kernels; FFTT_E_UNSUPPORTED
 *   where those do not apply).  The fixed point is unchanged; rel_tol still
 *   measures |J^T (d - J x)/sigma^2 - alpha x| relative to its start. */
typedef struct {
    int32_t method;
    int32_t prec;            /* fftt_precision */
    double alpha;
    double noise_sigma;
    int32_t max_iter;
    int32_t use_x0;
    double target_misfit;
    double rel_tol;
    int32_t use_graph;
    int32_t precond;         /* 0 none, 1 Jacobi (method 0) */
} fftt_solve_opts;

typedef struct {
    int32_t iters;
    double misfit;
    double rel_resid;
    double time_ms;
} fftt_solve_report;

fftt_status fftt_solve(fftt_ctx *ctx, const fftt_solve_opts *opts,
                       const void *d_obs, void *x, fftt_solve_report *rep);

/* Sensitivity coverage (Sec. III: the absolute values of the operator
 * summed over its rows) and the diagonal of the Gauss-Newton Hessian:
 *   kind 0: out_j = sum_b sum_i |J^b_ij|;   kind 1: out_j = sum_b sum_i (J^b_ij)^2
 * over every caller pair i (pairs sharing a row of J each count) and band b.
 * One J^T-like pass in FP32 with the current kernel evaluation (table or
 * series; prec FFTT_FP32 or FFTT_FP32_BF16TABLE selects the table), on the
 * LDS-staged kernels (FFTT_E_UNSUPPORTED where they do not apply, and for
 * FFTT_FP64).  out: device [N] FP32, inactive voxels 0.  Asynchronous. */
fftt_status fftt_coverage(fftt_ctx *ctx, fftt_precision prec, int32_t kind, void *out);

/* Low-rank eigen-decomposition of the Gauss-Newton Hessian of the misfit,
 * H = J^T J / sigma^2 summed over bands (eq. low_rank with Gamma_pr = I),
 * by a randomized range finder with q subspace iterations and a
 * Rayleigh-Ritz step (Halko, Martinsson & Tropp, SIAM Review 2011):
 * Q = orth(H omega), then q times Q = orth(H Q), then T = Q^T H Q = U Theta
 * U^T and the Ritz pairs (Theta, Q U).  orth keeps the directions whose
 * Gram eigenvalue exceeds 1e-24 (FP64) / 1e-12 (otherwise) of the largest,
 * so a sampled range of lower rank r yields r Ritz pairs; *rank_out (may be
 * NULL) returns r, and eigenvalues / vectors beyond r are 0.
 *   omega: device [l][N] start block (the caller's random numbers), in the
 *   operator's precision; 1 <= k <= l <= 512, 0 <= q <= 32.
 *   eigvals: host [k], descending; eigvecs: device [k][N], orthonormal.
 * Costs l + (q + 1) r applications of J and of J^T plus FP64 Gram matrices
 * of the blocks; synchronises the stream. */
fftt_status fftt_hessian_lowrank(fftt_ctx *ctx, fftt_precision prec, double noise_sigma,
                                 const void *omega, int32_t l, int32_t q, int32_t k,
                                 double *eigvals, void *eigvecs, int32_t *rank_out);

/* Gauss-Newton Hessian of the misfit applied to n_vec model vectors:
 * y_k = J^T J x_k / sigma^2 (bands summed; eq. resolution_2's H_misfit).
 * x, y: device [n_vec][N] in the precision's type.  FP32 / BF16-table
 * operators with 1 to 3 bands in 3D run as one batch (FFTT_TUNE_HESS_BATCHED):
 * per tile the products with all vectors are contractions on the BF16 matrix
 * cores, every FP32 operand split in two BF16 parts (hi hi + hi lo + lo hi,
 * FP32 accumulation; within 1e-5, norm-wise per vector, of the one-vector
 * path), partials summed per pair in FP64 in a fixed order.  Library
 * workspace: the per-(tile, pair) partials of a column batch, at most about
 * 8 GB (batches of fewer columns otherwise).  Asynchronous. */
fftt_status fftt_hessian_apply(fftt_ctx *ctx, fftt_precision prec, double noise_sigma,
                               const void *x, int32_t n_vec, void *y);

/* Diagonals of the low-rank posterior covariance and resolution matrix
 * (eq. posterior_app / resolution_app with Gamma_pr = I) from k eigenpairs
 * of H:  d_i = lambda_i / (lambda_i + alpha),
 *   var_j = (1 - sum_i d_i v_ij^2) / alpha,   res_j = sum_i d_i v_ij^2.
 * eigvals: host [k] (>= 0); eigvecs: device [k][N]; var_out, res_out: device
 * [N] or NULL (not both); buffers in the precision's type; alpha > 0.
 * Synchronises the stream. */
fftt_status fftt_lowrank_diag(fftt_ctx *ctx, fftt_precision prec, const double *eigvals,
                              const void *eigvecs, int32_t k, double alpha, void *var_out,
                              void *res_out);

/* Hessian point-spread functions (eq. resolution_2):
 * out[k] = J^T J e_{voxels[k]} / sigma^2, e_i = 1 m/s at voxel i, summed
 * over bands.
 *   voxels: host [n] active voxel indices;  out: device [n][N] (FP64 for
 *   FFTT_FP64, FP32 otherwise), overwritten.
 * FP32 / BF16-table precision with the staged kernels enabled (and the
 * tables plus n_tx * 512 bytes within LDS): all n in one batch -- the J^T
 * weights of every J e_k, then one launch that contracts the per-tile
 * kernel values with them on the matrix cores (BF16 with three-way split
 * operands for 1 to 3 bands, FP32 otherwise or with FFTT_TUNE_PSF_MATH = 1);
 * the batch requires (kernel pairs) * ceil32(n) < 2^30 and n < 2^22, else
 * FFTT_E_INVALID.  Otherwise one J and one J^T per voxel.  Library
 * workspace: nb * M * ceil32(n) floats.  Asynchronous except for the final
 * wait of the batched path. */
fftt_status fftt_psf(fftt_ctx *ctx, fftt_precision prec, const int64_t *voxels,
                     int32_t n, double noise_sigma, void *out);

/* Launch shape of the operator kernels (results do not depend on it):
 *   FFTT_TUNE_WAVES_PER_BLOCK: 4x4x4 voxel tiles (one wavefront each) per
 *     workgroup, sharing one LDS copy of the tables: 1, 2, 4, 8 or 16.
 *   FFTT_TUNE_UNROLL_JT / FFTT_TUNE_UNROLL_J: source-receiver entries per
 *     inner-loop step of the J^T / J kernel: 1, 2 or 4.
 *   FFTT_TUNE_SPLIT_JT / FFTT_TUNE_SPLIT_J: 0 = every wavefront owns a tile;
 *     1 = a workgroup owns a tile and its wavefronts split the tile's pairs.
 *   FFTT_TUNE_STAGED: 1 (default) = FP32/BF16 operators first evaluate the
 *     transducer distances of a tile into LDS (Q * 512 bytes plus the
 *     tables, see FFTT_TUNE_STAGED_BLOCK), 0 = never.  The staged kernels
 *     take fewer than 16384 transducers (their entry copies hold 14-bit
 *     transducer indices); with more, the per-wavefront kernels run.
 *   FFTT_TUNE_UNROLL_JT_STAGED / FFTT_TUNE_UNROLL_J_STAGED: unroll of those:
 *     1, 2, 4 or 8.
 *   FFTT_TUNE_STAGED_TABLE: table layout of the staged FP32 kernels:
 *     0 (default) = one float per node (4 bytes), 1 = (h_k, h_{k+1} - h_k)
 *     pairs (8 bytes per node, fewer instructions, more LDS).
 *   FFTT_TUNE_STAGED_BLOCK: the staged kernels stage transducers in aligned
 *     blocks of Q (a power of two: the smallest covering all transducers,
 *     halved until it fits LDS); a tile's entries are processed one block
 *     at a time, which requires every pair to lie in one block (else the
 *     per-wavefront kernels run).  0 (default) = automatic, otherwise an
 *     upper bound on Q (a power of two >= 16).
 *   FFTT_TUNE_KERNEL_EVAL: 0 (default) = the FP32 operators interpolate
 *     the table, 1 = they sum the bands' sine series (fftt_set_kernel_series).
 *   FFTT_TUNE_PSF_MATH: contraction of the batched FP32 / BF16-table PSFs:
 *     0 (default) = BF16 matrix cores with every FP32 operand split in two
 *     BF16 parts and three products (hi hi + hi lo + lo hi, FP32
 *     accumulation; 1 to 3 bands, 4 bands use FP32), 1 = FP32 matrix cores.
 *   FFTT_TUNE_HESS_BATCHED: 1 (default) = products of the Gauss-Newton
 *     Hessian with blocks of vectors (fftt_hessian_apply, the low-rank
 *     eigensolver) run batched on the matrix cores where they can (FP32 /
 *     BF16-table operators with table evaluation, 1 to 3 bands, 3D, LDS),
 *     0 = one J and one J^T per vector.
 *   FFTT_TUNE_RHS_BATCHED: 1 (default) = fftt_apply_J / fftt_apply_JT with
 *     n_rhs >= 8 run batched on the matrix cores where they can (as
 *     FFTT_TUNE_HESS_BATCHED), 0 = one launch per right-hand side.
 *   FFTT_TUNE_RECIPROCITY: 1 (default) = a pair (s, r) and its reverse
 *     (r, s) have the same row of J (source-receiver reciprocity of Sec. II;
 *     the detour and L are symmetric), so each unordered pair is evaluated
 *     once: J writes the row to both, J^T uses the summed data; 0 = every
 *     ordered pair is evaluated (only exact repeats share a row).  Outputs
 *     agree within rounding; changing it re-runs the set-up on next use.
 *   FFTT_TUNE_ENTRY_ORDER: 1 (default) = when every staged launch can stage
 *     all transducers at once (up to 1024), the staged J^T walks a copy of
 *     each tile's (tile, pair) list in which every pair is oriented towards
 *     its endpoint with more pairs in the tile and the list is grouped by
 *     that endpoint in fours, so that most half-steps share one staged
 *     source (the row of J is symmetric in source and receiver); 0 = a copy
 *     in pair order.  A change rebuilds the lists on next use.  J^T agrees
 *     within rounding (summation order).
 * FFTT_E_INVALID for other keys or values. */
enum { FFTT_TUNE_WAVES_PER_BLOCK = 0, FFTT_TUNE_UNROLL_JT = 1, FFTT_TUNE_UNROLL_J = 2,
       FFTT_TUNE_SPLIT_JT = 3, FFTT_TUNE_SPLIT_J = 4, FFTT_TUNE_STAGED = 5,
       FFTT_TUNE_UNROLL_JT_STAGED = 6, FFTT_TUNE_UNROLL_J_STAGED = 7,
       FFTT_TUNE_STAGED_TABLE = 8, FFTT_TUNE_RECIPROCITY = 9,
       FFTT_TUNE_STAGED_BLOCK = 10, FFTT_TUNE_KERNEL_EVAL = 11, FFTT_TUNE_PSF_MATH = 12,
       FFTT_TUNE_HESS_BATCHED = 13, FFTT_TUNE_RHS_BATCHED = 14, FFTT_TUNE_ENTRY_ORDER = 15 };
fftt_status fftt_set_tuning(fftt_ctx *ctx, int32_t key, int32_t value);

/* Current value of a tuning key (FFTT_E_INVALID for an unknown key). */
fftt_status fftt_get_tuning(fftt_ctx *ctx, int32_t key, int32_t *value);

/* Launch-shape autotuner: on the current geometry and tables, times the
 * J and J^T kernels (HIP events, library scratch vectors) under candidate
 * shapes -- staged or per-wavefront kernels, wavefronts per workgroup
 * (chosen for J + J^T together), unroll and split per operator, FP32 table
 * layout -- and keeps the fastest.  Stops trying new candidates after
 * max_seconds (> 0).  Results of the operators do not depend on the shape.
 * Synchronises the stream; FFTT_E_STATE before geometry and tables. */
fftt_status fftt_autotune(fftt_ctx *ctx, fftt_precision prec, double max_seconds);

/* Measurement aid.  With enable != 0 every launch of the main operator
 * kernels is bracketed by HIP events on the context's stream; enabling
 * clears the record.  fftt_kernel_time sums the recorded durations (ms) and
 * counts the launches of one kernel: which = 0 the J kernel, 1 the J^T
 * kernel, 2 the per-pair reduction of J, 3 the batched point-spread
 * functions (weights and matrix-core pass).  Synchronises the stream. */
fftt_status fftt_profile(fftt_ctx *ctx, int32_t enable);
fftt_status fftt_kernel_time(fftt_ctx *ctx, int32_t which, double *ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* FFTT_H */
