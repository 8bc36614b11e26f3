/*
 * polyeval -- evaluation of a sparse polynomial system and its Jacobian on an
 * AMD Instinct MI355X (gfx950), in complex double-double or complex FP64.
 *
 * The problem is the one of Verschelde & Yoffe, "Evaluating polynomials in
 * several variables and their derivatives on a GPU computing processor",
 * Section 2: a system f = (C, A) is a tuple of complex coefficients C and
 * exponent supports A, and each polynomial is
 *
 *     f_p(x) = sum_{a in A_p} c_a x^a,   x^a = x_1^{a_1} ... x_n^{a_n}.
 *
 * The library returns f(x) and the full Jacobian J(x) = (df_p/dx_i) at one
 * or many points, following the three stages of Section 2 and Section 3
 * (power table and common factors; Speelpenning products with forward and
 * backward partial products; coefficient multiplication and summation).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Complex numbers are passed as four planes of doubles (pe_cvec):
 *   value = (re_hi + re_lo) + i (im_hi + im_lo).  In PE_FP64 mode only the
 *   re_hi and im_hi planes are read and written; re_lo/im_lo may be NULL and
 *   are never touched.
 * - Points:   [n_points][n_vars]                      (per plane, row-major)
 *   Values:   [n_points][n_polys]
 *   Jacobian: [n_points][n_vars][n_polys]  i.e. column-major per point:
 *             entry (p, i) = df_p/dx_i at offset i*n_polys + p
 *             (the output order of Section 3.3: the values first, then the
 *             derivatives of all polynomials with respect to x_1, x_2, ...).
 * - Device pointers are owned by the caller; the library never frees them.
 *   Host arrays passed to pe_create_system are copied before it returns.
 * - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *   work on it and return without synchronizing, unless stated otherwise.
 * - Every entry point returns a pe_status.  On any status other than PE_OK a
 *   message is available from pe_last_error() (per thread).  No entry point
 *   aborts the process or throws across this interface.
 */
#ifndef POLYEVAL_H
#define POLYEVAL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pe_system_s *pe_system; /* opaque, immutable after creation */
typedef struct pe_batch_s *pe_batch;   /* opaque, several systems for one launch */

typedef enum { PE_FP64 = 0, PE_DD = 1 } pe_precision;

typedef enum { PE_NEWTON_MIXED = 0, PE_NEWTON_DD = 1 } pe_newton_mode;

typedef enum {
    PE_OK = 0,
    PE_EINVAL = 1,        /* invalid argument or system                     */
    PE_ENOMEM = 2,        /* device or host allocation failed               */
    PE_EDEVICE = 3,       /* a HIP call failed                              */
    PE_EUNSUPPORTED = 4,  /* valid input outside what the kernels support   */
    PE_ENOTCONVERGED = 5  /* Newton: some start did not converge            */
} pe_status;

typedef struct {
    double *re_hi;
    double *re_lo;
    double *im_hi;
    double *im_lo;
} pe_cvec;

/* Library version string. */
const char *pe_version(void);

/* Message for the last non-OK status returned on this thread. */
const char *pe_last_error(void);

/*
 * pe_create_system -- pack a system f = (C, A) (Section 2, equation (1)).
 *
 *   n_vars, n_polys  number of variables and of polynomials (both >= 1).
 *   n_monos          total number of monomials (>= 0).
 *   poly_start       [n_polys+1] host, CSR: polynomial p owns monomials
 *                    poly_start[p] .. poly_start[p+1]-1; poly_start[0] = 0,
 *                    non-decreasing, poly_start[n_polys] = n_monos.
 *   mono_start       [n_monos+1] host, CSR into pos/exp: monomial s owns
 *                    entries mono_start[s] .. mono_start[s+1]-1.  A monomial
 *                    may have no variables (a constant term).
 *   pos              [nnz] host, variable indices 0 <= pos < n_vars, strictly
 *                    increasing within a monomial (i_1 < i_2 < ... < i_k,
 *                    Section 2).
 *   exp              [nnz] host, exponents 1 <= exp <= 256.
 *   coef             [n_monos] host planes, finite complex dd coefficients.
 *                    Zero coefficients and repeated monomials are accepted
 *                    (they contribute 0, and add, respectively).
 *   out              receives the new handle.
 *
 * Uploads the packed tables to the current HIP device (synchronously).
 * Errors: PE_EINVAL (with a message naming the first bad entry), PE_ENOMEM,
 * PE_EDEVICE.
 */
pe_status pe_create_system(int32_t n_vars, int32_t n_polys, int64_t n_monos,
                           const int64_t *poly_start, const int64_t *mono_start,
                           const int32_t *pos, const int32_t *exp, pe_cvec coef,
                           pe_system *out);

/* Release a system and its device memory.  NULL is accepted. */
pe_status pe_destroy_system(pe_system sys);

/* Sizes of a system: any pointer may be NULL. */
pe_status pe_system_info(pe_system sys, int32_t *n_vars, int32_t *n_polys, int64_t *n_monos,
                         int32_t *max_k, int32_t *max_exp);

/*
 * pe_eval_jac -- values f(x) and Jacobians J(x) at n_points points
 * (Section 2: the three evaluation stages; Section 3: the kernels).
 *
 *   points    device planes [n_points][n_vars].
 *   out_f     device planes [n_points][n_polys].
 *   out_J     device planes [n_points][n_vars][n_polys]; if all four
 *             pointers are NULL the Jacobian is not computed.
 *   precision PE_DD (complex double-double) or PE_FP64 (complex double).
 *   stream    hipStream_t.
 *
 * Every output entry is written, including the exact zeros of the Jacobian
 * where a polynomial does not depend on a variable.  Results are
 * deterministic: the order of every summation is fixed by the system and
 * the schedule, not by timing.  Non-finite points propagate as IEEE values.
 * n_points == 0 is a no-op.  A schedule that splits each polynomial over
 * several workgroups (groups > 1) keeps their partial rows in a workspace
 * owned by the system, which grows on demand (the call then allocates and
 * synchronises the stream first); calls on one system that overlap in time
 * on different streams share it and race, calls on one stream are ordered.
 * Errors: PE_EINVAL (NULL handle, NULL required plane, n_points < 0),
 * PE_EUNSUPPORTED (the system does not fit the kernel limits: see the
 * message), PE_ENOMEM, PE_EDEVICE.
 */
pe_status pe_eval_jac(pe_system sys, int64_t n_points, pe_cvec points, pe_cvec out_f,
                      pe_cvec out_J, pe_precision precision, void *stream);

/*
 * pe_eval_jac_noalloc -- pe_eval_jac for callers that cannot allocate
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, layouts, kernels and results (bit for
 * bit) as pe_eval_jac under the same schedule.  It allocates nothing, on the
 * device or the host:
 *   - it uses only schedule tables that already exist: call pe_eval_jac
 *     once with the same n_points (or pin the schedule and call it once)
 *     beforehand, else PE_EUNSUPPORTED;
 *   - when the schedule splits a polynomial over workgroups (groups > 1),
 *     the partial rows live in a static device array of 32 MiB per device
 *     (n_points * n_polys * groups * (n_vars + 1) complex values, 32 bytes
 *     each in PE_DD and 16 in PE_FP64); a call that needs more returns
 *     PE_EUNSUPPORTED before launching anything.
 * Every call on one device shares that device's array and overwrites it
 * (each call writes every entry it reads back), so calls that overlap in
 * time on one device (different streams, or host threads) race; calls on
 * one stream are ordered and safe.  Errors as pe_eval_jac.
 */
pe_status pe_eval_jac_noalloc(pe_system sys, int64_t n_points, pe_cvec points, pe_cvec out_f,
                              pe_cvec out_J, pe_precision precision, void *stream);

/*
 * pe_eval_jac_qd -- f(x) and J(x) in complex quad-double arithmetic (about
 * 212 bits; the paper's Section 1 names quad double beside double double as
 * the extended precision for path tracking), by the same fused kernel as
 * pe_eval_jac.  Points and outputs are given as arrays of eight device plane
 * pointers, in the order re x0, re x1, re x2, re x3, im x0, im x1, im x2,
 * im x3 (a value is re x0 + re x1 + re x2 + re x3 + i (im x0 + ...)), with
 * the layouts of pe_eval_jac; out_J == NULL skips the Jacobian.  The
 * system's coefficients are the double-double ones given at creation.
 * Schedule: 256 threads, two or four variables per lane; each polynomial
 * and point takes one workgroup, or 2 or 4 when the (polynomial, point)
 * pairs are fewer than the device's compute units, their partial rows then
 * added by a second kernel through the system's workspace as in
 * pe_eval_jac.  Errors as pe_eval_jac; PE_EUNSUPPORTED when the
 * quad-double power table and staging area exceed 160 KiB of LDS.
 */
pe_status pe_eval_jac_qd(pe_system sys, int64_t n_points, const double *const *points,
                         double *const *out_f, double *const *out_J, void *stream);

/*
 * pe_eval_jac_paper_layout -- the same values and Jacobians as pe_eval_jac,
 * computed the way the paper organises its kernels (Section 3), for
 * comparison on the same GPU: a common-factor kernel (each thread raises its
 * variables to a_j - 1 by repeated multiplication and writes CF to global
 * memory, Section 3.1), a monomial kernel (Speelpenning partials times CF
 * times k + 1 coefficients prescaled by the exponents, scattered into a
 * dense array of n + 1 rows of m entries per polynomial with zeros where a
 * variable does not occur, Sections 3.2 and 3.3) and a summation kernel
 * (one thread per output adding its m entries in monomial order).  Same
 * arguments, layouts and errors as pe_eval_jac, plus PE_EUNSUPPORTED for
 * monomials of more than 32 variables.  The scratch (common factors and the
 * dense array, n_points * M * (n_vars + 2) complex values) is owned by the
 * system; a call with a different point count or precision than the
 * previous one lays it out again synchronously (not under stream capture).
 */
pe_status pe_eval_jac_paper_layout(pe_system sys, int64_t n_points, pe_cvec points,
                                   pe_cvec out_f, pe_cvec out_J, pe_precision precision,
                                   void *stream);

/*
 * pe_set_schedule -- pin the launch schedule used by pe_eval_jac for this
 * system: `lanes` lanes cooperate on one monomial (1, 2, 4, 8, 16 or 32),
 * `chunk_vars` variables per lane (2, 4 or 8), `threads` per workgroup
 * (64..1024, a multiple of 64) and `groups` workgroups per polynomial for a
 * point.  Passing 0 for these four restores their automatic selection.
 * `tile_points` (1..32, 0 = automatic) is the number of consecutive points
 * one workgroup evaluates together: a chunk of monomials is read from global
 * memory once and applied to every point of the tile, whose power tables and
 * accumulators all sit in LDS (Section 3.2 reads the variables once per
 * block; the tile extends that to the supports and coefficients).
 * `stage_buffers` (1 or 2, 0 = automatic) is the number of LDS areas the
 * terms are staged in before their summation: with two, the terms of the
 * next (chunk, point) item are computed while the previous item is summed,
 * with one barrier per item instead of two.  Errors: PE_EINVAL for values
 * outside these sets or lanes*chunk_vars below the largest monomial size of
 * the system; a tile that does not fit the LDS is reported by pe_eval_jac
 * (PE_EUNSUPPORTED).
 */
pe_status pe_set_schedule(pe_system sys, int32_t lanes, int32_t chunk_vars, int32_t threads,
                          int32_t groups, int32_t tile_points, int32_t stage_buffers);

/* The schedule pe_eval_jac would use for n_points points (same fields; any
 * output pointer may be NULL).  Asking for tile_points or stage_buffers
 * packs the schedule's tables if they do not exist yet (their sizes decide
 * what fits the LDS), with the figures of a double-double launch. */
pe_status pe_get_schedule(pe_system sys, int64_t n_points, int32_t *lanes, int32_t *chunk_vars,
                          int32_t *threads, int32_t *groups, int32_t *tile_points,
                          int32_t *stage_buffers);

/*
 * pe_newton -- Newton's method x <- x - J(x)^{-1} f(x) from n_starts starts
 * at once, the corrector the evaluation serves (the paper's abstract and
 * Section 1: evaluation dominates Newton's method for large systems).
 *
 *   n_starts    number of starts (>= 0); the system must be square.
 *   x           device dd planes [n_starts][n_vars]: starts on entry, final
 *               iterates on return.
 *   tol         stop a start when max_p |f_p(x)| < tol, the residual being
 *               evaluated in complex double-double (e.g. 1e-28).
 *   max_iter    maximal number of updates per start (>= 0).
 *   mode        PE_NEWTON_MIXED: Jacobian evaluated and factored in complex
 *               FP64 at x rounded to FP64, residual in complex dd rounded to
 *               FP64 as the right-hand side, update in dd (iterative
 *               refinement with a fresh Jacobian per step).
 *               PE_NEWTON_DD: f, J, elimination and update all in dd.
 *   res_out     device [n_starts]: max_p |f_p| at the returned x (NaN if
 *               non-finite).
 *   iters_out   device [n_starts]: updates applied.
 *   status_out  device [n_starts]: 0 converged, 1 iteration limit reached,
 *               2 zero pivot (singular Jacobian), 3 non-finite residual.
 *   stream      hipStream_t.
 *
 * Synchronous: returns when every start has stopped.  Workspace (Jacobians,
 * residuals, steps) is owned by the system and grows on demand.  Returns
 * PE_OK when every start converged, PE_ENOTCONVERGED (outputs written)
 * otherwise; PE_EINVAL for a non-square system or invalid arguments;
 * PE_EUNSUPPORTED when the power table does not fit in LDS; PE_ENOMEM;
 * PE_EDEVICE.
 */
pe_status pe_newton(pe_system sys, int64_t n_starts, pe_cvec x, double tol, int32_t max_iter,
                    pe_newton_mode mode, double *res_out, int32_t *iters_out, int32_t *status_out,
                    void *stream);

/*
 * pe_newton_qd -- pe_newton's mixed-precision mode one level up, to
 * quad-double accuracy (about 212 bits; the paper's Section 1 names quad
 * double beside double double as the extended precision of path tracking):
 * the Jacobian is evaluated and factored in complex FP64 at x rounded to
 * FP64, the residual f(x) is evaluated in complex quad-double and rounded to
 * FP64 as the right-hand side, and x is updated in quad-double.  Each step
 * gains about the digits the FP64 solve gets right, so from a start good to
 * 1e-6 about five steps reach 1e-60.
 *
 *   x           eight device plane pointers [n_starts][n_vars] in the order
 *               of pe_eval_jac_qd (re x0..x3, im x0..x3): starts on entry,
 *               final iterates on return.
 *   tol         stop a start when max_p |f_p(x)| < tol, the residual in
 *               complex quad-double (e.g. 1e-56; the residual's own rounding
 *               is about 1e-63 times the sum of the magnitudes of a
 *               polynomial's terms).
 *   max_iter, res_out, iters_out, status_out, stream: as pe_newton.
 *
 * Synchronous, with pe_newton's statuses and errors; PE_EUNSUPPORTED also
 * when the quad-double power table x^1 .. x^d of n_vars variables (64 bytes
 * per entry) exceeds 160 KiB of LDS.  The system's coefficients are the
 * double-double ones given at creation.
 */
pe_status pe_newton_qd(pe_system sys, int64_t n_starts, double *const *x, double tol,
                       int32_t max_iter, double *res_out, int32_t *iters_out, int32_t *status_out,
                       void *stream);

/*
 * Path tracking: finding the roots of a square system by continuation, the
 * use the paper's introduction names for fast evaluation and Newton's
 * method (Section 1).  The homotopy is the total-degree one,
 *
 *     H(x, t) = (1 - t) * gamma * G(x) + t * F(x),  G_i(x) = x_i^{d_i} - 1,
 *
 * with d_i the total degree of f_i (the largest sum of exponents of its
 * monomials; every d_i must be >= 1), from the d_1 * ... * d_n start
 * solutions of G at t = 0 to the roots of F at t = 1.
 *
 * pe_start_solutions -- x <- start solutions first .. first+n_paths-1 of G:
 * path q has mixed-radix digits k_i in base d_i (the digit of x_0 varying
 * fastest, q taken modulo d_1 * ... * d_n) and x_i = exp(2 pi i k_i / d_i).
 * x: device dd planes [n_paths][n_vars] (low words written 0).
 * Errors: PE_EINVAL (non-square system, a polynomial of degree 0, first < 0,
 * n_paths < 0, NULL plane).
 */
pe_status pe_start_solutions(pe_system sys, int64_t first, int64_t n_paths, pe_cvec x,
                             void *stream);

typedef struct {
    double gamma_re, gamma_im; /* gamma (nonzero; a random point of the unit
                                  circle keeps the paths regular) */
    double h_init;             /* first step in t, in (0, 1] (e.g. 0.02) */
    double h_min;              /* a path stops when its step falls below (e.g. 1e-10) */
    double h_max;              /* largest step, >= h_init (e.g. 0.1) */
    double corr_tol;           /* the corrector accepts when its last Newton step
                                  has max |dx_i| <= corr_tol (1 + max |x_i|) (e.g. 1e-10) */
    int32_t corr_iters;        /* Newton iterations per corrector, >= 1 (e.g. 4) */
    int32_t max_steps;         /* step attempts per path, >= 1 (e.g. 4000) */
    double end_tol;            /* endgame: mixed-precision Newton (pe_newton's
                                  PE_NEWTON_MIXED) at t = 1 until max_p |f_p| <
                                  end_tol in complex dd; 0 skips it (e.g. 1e-28) */
    int32_t end_iters;         /* endgame iteration limit, >= 0 (e.g. 8) */
} pe_track_params;

/*
 * pe_track -- track n_paths paths of the homotopy from t = 0 to t = 1.
 *
 *   x          device dd planes [n_paths][n_vars]: start solutions of G on
 *              entry (only the high words are read), end points on return.
 *   params     host, see pe_track_params.
 *   t_out      device [n_paths]: the t each path reached.
 *   steps_out  device [n_paths]: step attempts (accepted and rejected).
 *   status_out device [n_paths]: 0 reached t = 1 (and, with an endgame,
 *              converged to end_tol), 1 step size fell below h_min,
 *              2 zero pivot (singular Jacobian), 3 non-finite values,
 *              4 step limit reached, 5 endgame did not converge.
 *   res_out    device [n_paths]: max_p |f_p| at the returned x after the
 *              endgame, NaN for paths without one.
 *
 * Tracking is in complex FP64: every round of the loop evaluates F and its
 * Jacobian at each running path's x (pe_eval_jac in PE_FP64), solves with
 * the homotopy's Jacobian H_x = t J_F + (1 - t) gamma diag(d_i x_i^{d_i-1})
 * (the batched elimination of pe_newton) and applies one step of the path:
 * an Euler predictor along dx/dt = -H_x^{-1} (F - gamma G), then Newton
 * corrector iterations on H(., t + h).  A step is accepted when its
 * corrector converges within corr_iters iterations, and the step size
 * doubles after three accepted steps in a row (up to h_max); otherwise the
 * path returns to its last accepted point with half the step.
 * Synchronous (the host reads the count of running paths every round), so
 * it cannot be captured in a graph.  Workspace is owned by the system and
 * grows on demand.  Returns PE_OK when every path has status 0,
 * PE_ENOTCONVERGED (outputs written) otherwise; PE_EINVAL for invalid
 * arguments, PE_EUNSUPPORTED when the elimination panel or the residual's
 * power table does not fit in LDS, PE_ENOMEM, PE_EDEVICE.
 */
pe_status pe_track(pe_system sys, int64_t n_paths, pe_cvec x, const pe_track_params *params,
                   double *t_out, int32_t *steps_out, int32_t *status_out, double *res_out,
                   void *stream);

/*
 * Batches: several systems (of any shapes) evaluated in one persistent
 * launch.  The systems must outlive the batch and stay on one device.
 *
 * pe_create_batch -- a batch over systems[0 .. count-1] (not owned).
 */
pe_status pe_create_batch(const pe_system *systems, int32_t count, pe_batch *out);

/* Release a batch (the systems are untouched).  NULL is accepted. */
pe_status pe_destroy_batch(pe_batch batch);

/*
 * pe_batch_layout -- element offsets of each system's block in the
 * concatenated buffers of pe_eval_jac_batch, for points_per_system[i] points
 * of system i: points_offset[i] (in [P_i][n_i] blocks), f_offset[i]
 * ([P_i][n_polys_i]) and J_offset[i] ([P_i][n_i][n_polys_i]); entry `count`
 * holds the totals.  Each output array has count+1 entries and may be NULL.
 */
pe_status pe_batch_layout(pe_batch batch, const int64_t *points_per_system,
                          int64_t *points_offset, int64_t *f_offset, int64_t *J_offset);

/*
 * pe_eval_jac_batch -- f and J of every system at its points, in one launch
 * of the persistent batch kernel (the three stages of Section 2 for every
 * system; Section 3's kernels fused).
 *
 *   points_per_system  host [count]: number of points of each system (>= 0).
 *   points, out_f, out_J  device planes, the systems' blocks concatenated in
 *                      batch order at the offsets of pe_batch_layout; out_J
 *                      all-NULL skips the Jacobians.
 *
 * The first call for given point counts (or after tuning) builds and uploads
 * the task list synchronously; later calls with the same counts only launch
 * the kernel, allocate nothing and may be captured in a hipGraph.  Results
 * equal pe_eval_jac's on each system up to the summation order.
 */
pe_status pe_eval_jac_batch(pe_batch batch, const int64_t *points_per_system, pe_cvec points,
                            pe_cvec out_f, pe_cvec out_J, pe_precision precision, void *stream);

/* The batch schedule in use: variables per lane, workgroup size, multiple of
 * the minimal lanes per monomial, target terms per task. */
pe_status pe_batch_config(pe_batch batch, int32_t *chunk_vars, int32_t *threads,
                          int32_t *lanes_mult, int32_t *task_terms);

/*
 * pe_autotune_batch -- choose the batch schedule (variables per lane,
 * workgroup size, lanes per monomial i.e. monomials per wavefront, task
 * size) by timing candidates on the given buffers (their contents are
 * overwritten), and keep the fastest.  If cache_path is not NULL the choice
 * is looked up in / appended to that text file, keyed by the shapes.
 * Synchronous.
 */
pe_status pe_autotune_batch(pe_batch batch, const int64_t *points_per_system, pe_cvec points,
                            pe_cvec out_f, pe_cvec out_J, pe_precision precision, void *stream,
                            const char *cache_path);

/*
 * pe_autotune_system -- the same for pe_eval_jac on one system at n_points
 * points: times schedules (lanes per monomial, variables per lane, threads,
 * groups) with one-point tiles and one staging buffer, then the tile sizes
 * 1, 2, 4, 8 and one or two staging buffers for the three fastest, and pins
 * the fastest with pe_set_schedule.  Synchronous.
 */
pe_status pe_autotune_system(pe_system sys, int64_t n_points, pe_cvec points, pe_cvec out_f,
                             pe_cvec out_J, pe_precision precision, void *stream,
                             const char *cache_path);

#ifdef __cplusplus
}
#endif

#endif /* POLYEVAL_H */
