// Newton corrector on top of the evaluator (C interface).
//
// Newton's method is where the evaluation of f and its Jacobian is the
// costly step (the paper's abstract and Section 1).  Two modes:
//   PE_NEWTON_MIXED  the Jacobian is evaluated and factored in complex FP64
//                    at x rounded to FP64; the residual f(x) is evaluated in
//                    complex double-double (the accuracy-critical step) and
//                    rounded to FP64 as the right-hand side; x is updated in
//                    double-double.  This is iterative refinement with a
//                    fresh Jacobian per step.
//   PE_NEWTON_DD     textbook Newton entirely in complex double-double: f
//                    and J from the dd evaluator, dd elimination, dd update.
// Both stop a start when max_p |f_p(x)| < tol (residual measured in dd).
// pe_newton_qd is the mixed mode one level up: FP64 Jacobian and
// elimination, residual and x in complex quad-double, so the same FP64
// solves refine x to quad-double accuracy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "polyeval.h"
#include "internal.hpp"
#include "newton.hpp"

using namespace pe;

namespace {

hipError_t grow(DevBuf &b, size_t bytes)
{
    if (b.bytes >= bytes) return hipSuccess;
    return b.alloc(bytes);
}

}  // namespace

namespace pe {

// kind 0: mixed (FP64 J and elimination, dd residual and x); 1: all dd;
// 2: mixed with quad-double residual and x (x has 8 planes).
static pe_status newton_core(System *S, int64_t n_starts, double *const *x, int kind, double tol,
                             int32_t max_iter, double *res_out, int32_t *iters_out,
                             int32_t *status_out, hipStream_t hs, bool init)
{
    const bool mixed = kind != 1;
    const bool qd = kind == 2;
    const int n = S->n_vars;
    const size_t SN = (size_t)n_starts * n;
    const size_t SNN = SN * n;
    const int jw = mixed ? 2 : 4;  // doubles per Jacobian entry
    const int rw = qd ? 8 : 4;     // doubles per residual entry
    hipError_t e = hipSuccess;
    if ((e = grow(S->nw_J, SNN * jw * sizeof(double))) != hipSuccess ||
        (e = grow(S->nw_r, SN * rw * sizeof(double))) != hipSuccess ||
        (e = grow(S->nw_d, SN * jw * sizeof(double))) != hipSuccess ||
        (e = grow(S->nw_f64, SN * 2 * sizeof(double))) != hipSuccess ||
        (e = grow(S->nw_counter, sizeof(int32_t))) != hipSuccess)
        return hip_fail(e, "allocating the Newton workspace");

    double *Jb = (double *)S->nw_J.ptr;
    double *rb = (double *)S->nw_r.ptr;
    double *db = (double *)S->nw_d.ptr;
    double *fb = (double *)S->nw_f64.ptr;
    int32_t *counter = (int32_t *)S->nw_counter.ptr;
    double *Jp[4], *dp[4];
    if (mixed) {
        double *Jq[4] = {Jb, nullptr, Jb + SNN, nullptr};
        double *dq[4] = {db, nullptr, db + SN, nullptr};
        std::copy(Jq, Jq + 4, Jp);
        std::copy(dq, dq + 4, dp);
    } else {
        double *Jq[4] = {Jb, Jb + SNN, Jb + 2 * SNN, Jb + 3 * SNN};
        double *dq[4] = {db, db + SN, db + 2 * SN, db + 3 * SN};
        std::copy(Jq, Jq + 4, Jp);
        std::copy(dq, dq + 4, dp);
    }
    // residual planes; the checks and the FP64 right-hand side read the
    // leading words through a dd-shaped view (planes 0 and 2 of it)
    double *rp[8];
    for (int q = 0; q < rw; ++q) rp[q] = rb + q * SN;
    const double *rview[4] = {rp[0], rp[1], qd ? rp[4] : rp[2], qd ? rp[5] : rp[3]};
    const double *dpc[4] = {dp[0], dp[1], dp[2], dp[3]};
    double *fp64[4] = {fb, nullptr, fb + SN, nullptr};
    // x seen as dd (for the evaluations): re x0, re x1, im x0, im x1
    const double *xview[4] = {x[0], x[1], qd ? x[4] : x[2], qd ? x[5] : x[3]};

    ResidArgs ra{};
    ra.n_vars = n;
    ra.n_polys = S->n_polys;
    ra.R = S->max_exp;
    ra.poly_start = (const int64_t *)S->d_poly_start.ptr;
    ra.mono_start = (const int32_t *)S->d_mono_start.ptr;
    ra.word = (const uint32_t *)S->d_word.ptr;
    ra.coef = (const double *)S->coef.ptr;
    ra.n_points = n_starts;
    for (int q = 0; q < rw; ++q) {
        ra.x[q] = x[q];
        ra.f[q] = rp[q];
    }
    ra.status = status_out;
    if (!resid_fits(qd ? 2 : 1, n, ra.R))
        return fail(PE_EUNSUPPORTED, "power table of the residual does not fit in LDS");
    if (!lu_solve_fits(mixed ? 0 : 1, n))
        return fail(PE_EUNSUPPORTED, "the elimination panel (n = %d) does not fit in LDS", n);

    if (init && (e = launch_newton_init(n_starts, status_out, iters_out, hs)) != hipSuccess)
        return hip_fail(e, "starting Newton");
    for (;;) {
        pe_status st;
        if (mixed) {
            if ((e = launch_resid(ra, qd ? 2 : 1, hs)) != hipSuccess)
                return hip_fail(e, "residual kernel");
        } else {
            st = S->eval_locked(n_starts, xview, rp, Jp, true, hs, status_out);
            if (st != PE_OK) return st;
        }
        if ((e = hipMemsetAsync(counter, 0, sizeof(int32_t), hs)) != hipSuccess)
            return hip_fail(e, "clearing the counter");
        if ((e = launch_check(n_starts, S->n_polys, rview, tol, max_iter, res_out, iters_out,
                              status_out, counter, hs)) != hipSuccess)
            return hip_fail(e, "residual check");
        int32_t running = 0;
        if ((e = hipMemcpyAsync(&running, counter, sizeof running, hipMemcpyDeviceToHost, hs)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(hs)) != hipSuccess)
            return hip_fail(e, "reading the running count");
        if (running == 0) break;
        if (mixed) {
            st = S->eval_locked(n_starts, xview, fp64, Jp, false, hs, status_out);
            if (st != PE_OK) return st;
            if ((e = launch_lu_solve(0, n_starts, n, Jp, rview, dp, status_out, hs)) != hipSuccess)
                return hip_fail(e, "FP64 solve");
            if ((e = launch_update(qd ? 2 : 0, n_starts, n, x, dpc, status_out, iters_out, hs)) !=
                hipSuccess)
                return hip_fail(e, "update");
        } else {
            if ((e = launch_lu_solve(1, n_starts, n, Jp, rview, dp, status_out, hs)) != hipSuccess)
                return hip_fail(e, "dd solve");
            if ((e = launch_update(1, n_starts, n, x, dpc, status_out, iters_out, hs)) != hipSuccess)
                return hip_fail(e, "update");
        }
    }
    std::vector<int32_t> stat((size_t)n_starts);
    if ((e = hipMemcpyAsync(stat.data(), status_out, stat.size() * sizeof(int32_t),
                            hipMemcpyDeviceToHost, hs)) != hipSuccess ||
        (e = hipStreamSynchronize(hs)) != hipSuccess)
        return hip_fail(e, "reading the statuses");
    int64_t bad = 0;
    for (int32_t v : stat) bad += (v != 0);
    if (bad) return fail(PE_ENOTCONVERGED, "%lld of %lld starts did not converge", (long long)bad,
                         (long long)n_starts);
    return PE_OK;
}

pe_status newton_run(System *S, int64_t n_starts, pe_cvec x, double tol, int32_t max_iter,
                     bool mixed, double *res_out, int32_t *iters_out, int32_t *status_out,
                     hipStream_t hs, bool init)
{
    double *xp[4] = {x.re_hi, x.re_lo, x.im_hi, x.im_lo};
    return newton_core(S, n_starts, xp, mixed ? 0 : 1, tol, max_iter, res_out, iters_out,
                       status_out, hs, init);
}

}  // namespace pe

extern "C" pe_status pe_newton(pe_system sys, int64_t n_starts, pe_cvec x, double tol,
                               int32_t max_iter, pe_newton_mode mode, double *res_out,
                               int32_t *iters_out, int32_t *status_out, void *stream)
{
    if (!sys) return fail(PE_EINVAL, "NULL system");
    System *S = reinterpret_cast<System *>(sys);
    if (S->n_vars != S->n_polys)
        return fail(PE_EINVAL, "Newton needs a square system (n_vars %d != n_polys %d)", S->n_vars,
                    S->n_polys);
    if (n_starts < 0) return fail(PE_EINVAL, "n_starts < 0");
    if (!(tol > 0.0)) return fail(PE_EINVAL, "tol must be > 0");
    if (max_iter < 0) return fail(PE_EINVAL, "max_iter must be >= 0");
    if (mode != PE_NEWTON_MIXED && mode != PE_NEWTON_DD) return fail(PE_EINVAL, "unknown mode");
    if (n_starts == 0) return PE_OK;
    if (!x.re_hi || !x.re_lo || !x.im_hi || !x.im_lo) return fail(PE_EINVAL, "a plane of x is NULL");
    if (!res_out || !iters_out || !status_out) return fail(PE_EINVAL, "an output array is NULL");
    if (n_starts > 0x7FFFFFFF) return fail(PE_EUNSUPPORTED, "too many starts");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != S->device)
        return fail(PE_EINVAL, "the current device is not the system's device");

    std::lock_guard<std::mutex> lock(S->mu);
    return newton_run(S, n_starts, x, tol, max_iter, mode == PE_NEWTON_MIXED, res_out, iters_out,
                      status_out, reinterpret_cast<hipStream_t>(stream), true);
}

extern "C" pe_status pe_newton_qd(pe_system sys, int64_t n_starts, double *const *x, double tol,
                                  int32_t max_iter, double *res_out, int32_t *iters_out,
                                  int32_t *status_out, void *stream)
{
    if (!sys) return fail(PE_EINVAL, "NULL system");
    System *S = reinterpret_cast<System *>(sys);
    if (S->n_vars != S->n_polys)
        return fail(PE_EINVAL, "Newton needs a square system (n_vars %d != n_polys %d)", S->n_vars,
                    S->n_polys);
    if (n_starts < 0) return fail(PE_EINVAL, "n_starts < 0");
    if (!(tol > 0.0)) return fail(PE_EINVAL, "tol must be > 0");
    if (max_iter < 0) return fail(PE_EINVAL, "max_iter must be >= 0");
    if (n_starts == 0) return PE_OK;
    if (!x) return fail(PE_EINVAL, "NULL plane array");
    for (int q = 0; q < 8; ++q)
        if (!x[q]) return fail(PE_EINVAL, "plane %d of x is NULL", q);
    if (!res_out || !iters_out || !status_out) return fail(PE_EINVAL, "an output array is NULL");
    if (n_starts > 0x7FFFFFFF) return fail(PE_EUNSUPPORTED, "too many starts");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != S->device)
        return fail(PE_EINVAL, "the current device is not the system's device");

    std::lock_guard<std::mutex> lock(S->mu);
    return newton_core(S, n_starts, x, 2, tol, max_iter, res_out, iters_out, status_out,
                       reinterpret_cast<hipStream_t>(stream), true);
}
