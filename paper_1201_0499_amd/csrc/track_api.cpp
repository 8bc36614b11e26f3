// Path tracker on top of the evaluator and the Newton corrector (C
// interface); the kernels and the method are described in track.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "polyeval.h"
#include "internal.hpp"
#include "newton.hpp"
#include "track.hpp"

using namespace pe;

namespace {

hipError_t grow(DevBuf &b, size_t bytes)
{
    if (b.bytes >= bytes) return hipSuccess;
    return b.alloc(bytes);
}

// Total degrees of the polynomials, uploaded once; PE_EINVAL if one is 0.
pe_status upload_degrees(System *S)
{
    if (S->tk_deg.ptr) return PE_OK;
    std::vector<int32_t> deg((size_t)S->n_polys, 0);
    for (int p = 0; p < S->n_polys; ++p) {
        int64_t best = 0;
        for (int64_t s = S->poly_start[p]; s < S->poly_start[p + 1]; ++s) {
            int64_t d = 0;
            for (int64_t j = S->mono_start[s]; j < S->mono_start[s + 1]; ++j) d += S->exp[(size_t)j];
            best = std::max(best, d);
        }
        if (best < 1)
            return fail(PE_EINVAL, "polynomial %d has total degree 0: no start system", p);
        if (best > 0x7FFFFFFF) return fail(PE_EUNSUPPORTED, "polynomial %d: degree too large", p);
        deg[(size_t)p] = (int32_t)best;
    }
    hipError_t e = S->tk_deg.upload(deg.data(), deg.size() * sizeof(int32_t));
    if (e != hipSuccess) return hip_fail(e, "uploading the degrees");
    return PE_OK;
}

pe_status check_system(pe_system sys, System **out)
{
    if (!sys) return fail(PE_EINVAL, "NULL system");
    System *S = reinterpret_cast<System *>(sys);
    if (S->n_vars != S->n_polys)
        return fail(PE_EINVAL, "path tracking needs a square system (n_vars %d != n_polys %d)",
                    S->n_vars, S->n_polys);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != S->device)
        return fail(PE_EINVAL, "the current device is not the system's device");
    *out = S;
    return PE_OK;
}

}  // namespace

extern "C" pe_status pe_start_solutions(pe_system sys, int64_t first, int64_t n_paths, pe_cvec x,
                                        void *stream)
{
    System *S = nullptr;
    pe_status st = check_system(sys, &S);
    if (st != PE_OK) return st;
    if (first < 0 || n_paths < 0) return fail(PE_EINVAL, "first and n_paths must be >= 0");
    if (n_paths == 0) return PE_OK;
    if (!x.re_hi || !x.re_lo || !x.im_hi || !x.im_lo) return fail(PE_EINVAL, "a plane of x is NULL");
    std::lock_guard<std::mutex> lock(S->mu);
    if ((st = upload_degrees(S)) != PE_OK) return st;
    double *xp[4] = {x.re_hi, x.re_lo, x.im_hi, x.im_lo};
    hipError_t e = launch_track_start(first, n_paths, S->n_vars, (const int32_t *)S->tk_deg.ptr, xp,
                                      reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "start solutions");
    return PE_OK;
}

extern "C" pe_status pe_track(pe_system sys, int64_t n_paths, pe_cvec x,
                              const pe_track_params *prm, double *t_out, int32_t *steps_out,
                              int32_t *status_out, double *res_out, void *stream)
{
    System *S = nullptr;
    pe_status st = check_system(sys, &S);
    if (st != PE_OK) return st;
    if (!prm) return fail(PE_EINVAL, "NULL params");
    if (n_paths < 0) return fail(PE_EINVAL, "n_paths < 0");
    if (n_paths > 0x7FFFFFFF) return fail(PE_EUNSUPPORTED, "too many paths");
    const pe_track_params P = *prm;
    if (!(std::isfinite(P.gamma_re) && std::isfinite(P.gamma_im)) ||
        (P.gamma_re == 0.0 && P.gamma_im == 0.0))
        return fail(PE_EINVAL, "gamma must be finite and nonzero");
    if (!(P.h_init > 0.0 && P.h_init <= 1.0)) return fail(PE_EINVAL, "h_init must be in (0, 1]");
    if (!(P.h_min > 0.0 && P.h_min <= P.h_init)) return fail(PE_EINVAL, "h_min must be in (0, h_init]");
    if (!(P.h_max >= P.h_init && std::isfinite(P.h_max))) return fail(PE_EINVAL, "h_max must be >= h_init");
    if (!(P.corr_tol > 0.0)) return fail(PE_EINVAL, "corr_tol must be > 0");
    if (P.corr_iters < 1) return fail(PE_EINVAL, "corr_iters must be >= 1");
    if (P.max_steps < 1) return fail(PE_EINVAL, "max_steps must be >= 1");
    if (!(P.end_tol >= 0.0)) return fail(PE_EINVAL, "end_tol must be >= 0");
    if (P.end_iters < 0) return fail(PE_EINVAL, "end_iters must be >= 0");
    if (n_paths == 0) return PE_OK;
    if (!x.re_hi || !x.re_lo || !x.im_hi || !x.im_lo) return fail(PE_EINVAL, "a plane of x is NULL");
    if (!t_out || !steps_out || !status_out || !res_out)
        return fail(PE_EINVAL, "an output array is NULL");

    std::lock_guard<std::mutex> lock(S->mu);
    if ((st = upload_degrees(S)) != PE_OK) return st;
    const int n = S->n_vars;
    if (!lu_solve_fits(0, n))
        return fail(PE_EUNSUPPORTED, "the elimination panel (n = %d) does not fit in LDS", n);
    if (P.end_tol > 0.0 && (size_t)S->max_exp * (n + 1) * 32 > kMaxLds)
        return fail(PE_EUNSUPPORTED, "power table of the endgame residual does not fit in LDS");
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    const size_t PN = (size_t)n_paths * n, PNN = PN * n, NP = (size_t)n_paths;
    hipError_t e = hipSuccess;
    // state: t, t1, h (doubles), then phase, succ, tracked, end iterations (int32)
    const size_t state_bytes = NP * (3 * sizeof(double) + 4 * sizeof(int32_t));
    if ((e = grow(S->nw_J, PNN * 2 * sizeof(double))) != hipSuccess ||
        (e = grow(S->nw_r, PN * 4 * sizeof(double))) != hipSuccess ||
        (e = grow(S->nw_d, PN * 2 * sizeof(double))) != hipSuccess ||
        (e = grow(S->nw_f64, PN * 2 * sizeof(double))) != hipSuccess ||
        (e = grow(S->nw_counter, sizeof(int32_t))) != hipSuccess ||
        (e = grow(S->tk_xs, PN * 2 * sizeof(double))) != hipSuccess ||
        (e = grow(S->tk_state, state_bytes)) != hipSuccess)
        return hip_fail(e, "allocating the tracker workspace");

    double *Jb = (double *)S->nw_J.ptr, *rb = (double *)S->nw_r.ptr;
    double *db = (double *)S->nw_d.ptr, *fb = (double *)S->nw_f64.ptr;
    double *xsb = (double *)S->tk_xs.ptr;
    double *tb = (double *)S->tk_state.ptr;
    int32_t *ib = (int32_t *)(tb + 3 * NP);
    int32_t *counter = (int32_t *)S->nw_counter.ptr;

    TrackArgs a{};
    a.n_paths = n_paths;
    a.n = n;
    a.gamma_re = P.gamma_re;
    a.gamma_im = P.gamma_im;
    a.deg = (const int32_t *)S->tk_deg.ptr;
    a.h_min = P.h_min;
    a.h_max = P.h_max;
    a.corr_tol = P.corr_tol;
    a.corr_iters = P.corr_iters;
    a.max_steps = P.max_steps;
    a.x[0] = x.re_hi;
    a.x[1] = x.im_hi;
    a.f[0] = fb;
    a.f[1] = fb + PN;
    a.J[0] = Jb;
    a.J[1] = Jb + PNN;
    a.r[0] = rb;
    a.r[1] = rb + PN;
    a.d[0] = db;
    a.d[1] = db + PN;
    a.xs[0] = xsb;
    a.xs[1] = xsb + PN;
    a.t = tb;
    a.t1 = tb + NP;
    a.h = tb + 2 * NP;
    a.phase = ib;
    a.succ = ib + NP;
    int32_t *tracked = ib + 2 * NP;
    int32_t *end_iters = ib + 3 * NP;
    a.steps = steps_out;
    a.status = status_out;
    a.running = counter;

    const double *xpc[4] = {x.re_hi, x.re_lo, x.im_hi, x.im_lo};
    double *fq[4] = {fb, nullptr, fb + PN, nullptr};
    double *Jq[4] = {Jb, nullptr, Jb + PNN, nullptr};
    const double *rq[4] = {rb, nullptr, rb + PN, nullptr};
    double *dq[4] = {db, nullptr, db + PN, nullptr};
    double *xlo[2] = {x.re_lo, x.im_lo};

    if ((e = launch_track_init(a, P.h_init, xlo, hs)) != hipSuccess) return hip_fail(e, "tracker init");
    // every step attempt takes at most 1 + corr_iters rounds
    const int64_t max_rounds = (int64_t)P.max_steps * (1 + P.corr_iters) + 2;
    for (int64_t round = 0; round < max_rounds; ++round) {
        st = S->eval_locked(n_paths, xpc, fq, Jq, false, hs, status_out);
        if (st != PE_OK) return st;
        if ((e = launch_track_homotopy(a, hs)) != hipSuccess) return hip_fail(e, "homotopy kernel");
        if ((e = launch_lu_solve(0, n_paths, n, Jq, rq, dq, status_out, hs)) != hipSuccess)
            return hip_fail(e, "tracker solve");
        if ((e = hipMemsetAsync(counter, 0, sizeof(int32_t), hs)) != hipSuccess)
            return hip_fail(e, "clearing the counter");
        if ((e = launch_track_step(a, hs)) != hipSuccess) return hip_fail(e, "step kernel");
        int32_t running = 0;
        if ((e = hipMemcpyAsync(&running, counter, sizeof running, hipMemcpyDeviceToHost, hs)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(hs)) != hipSuccess)
            return hip_fail(e, "reading the running count");
        if (running == 0) break;
    }
    // NaN residuals unless an endgame writes them
    if ((e = hipMemsetAsync(res_out, 0xFF, NP * sizeof(double), hs)) != hipSuccess)
        return hip_fail(e, "clearing the residuals");
    if (P.end_tol > 0.0) {
        if ((e = launch_track_endgame(n_paths, tracked, status_out, hs)) != hipSuccess ||
            (e = hipMemsetAsync(end_iters, 0, NP * sizeof(int32_t), hs)) != hipSuccess)
            return hip_fail(e, "starting the endgame");
        st = newton_run(S, n_paths, x, P.end_tol, P.end_iters, true, res_out, end_iters, status_out,
                        hs, false);
        if (st != PE_OK && st != PE_ENOTCONVERGED) return st;
        if ((e = launch_track_end(n_paths, tracked, status_out, hs)) != hipSuccess)
            return hip_fail(e, "ending the endgame");
    }
    if ((e = hipMemcpyAsync(t_out, a.t, NP * sizeof(double), hipMemcpyDeviceToDevice, hs)) !=
        hipSuccess)
        return hip_fail(e, "copying t");
    std::vector<int32_t> stat(NP);
    if ((e = hipMemcpyAsync(stat.data(), status_out, NP * sizeof(int32_t), hipMemcpyDeviceToHost,
                            hs)) != hipSuccess ||
        (e = hipStreamSynchronize(hs)) != hipSuccess)
        return hip_fail(e, "reading the statuses");
    int64_t bad = 0;
    for (int32_t v : stat) bad += (v != 0);
    if (bad)
        return fail(PE_ENOTCONVERGED, "%lld of %lld paths did not reach a root",
                    (long long)bad, (long long)n_paths);
    return PE_OK;
}
