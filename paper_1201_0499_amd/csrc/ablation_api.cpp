// The paper's three-kernel evaluation behind the C interface (see
// ablation.hip): same inputs, outputs and checks as pe_eval_jac.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "polyeval.h"
#include "ablation.hpp"
#include "dd.hpp"
#include "internal.hpp"

using namespace pe;

namespace {

// Per-system tables of the three-kernel path: polynomial of each monomial
// and the k + 1 prescaled coefficients (c a_j, then c) of each monomial.
pe_status upload_tables(System *S)
{
    if (S->ab_mono_poly.ptr || S->n_monos == 0) return PE_OK;
    const int64_t M = S->n_monos;
    std::vector<int32_t> mono_poly((size_t)M), start((size_t)M);
    std::vector<double> pc;
    std::vector<double> coef((size_t)M * 4);
    hipError_t e = hipMemcpy(coef.data(), S->coef.ptr, coef.size() * sizeof(double),
                             hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "reading the coefficients");
    for (int p = 0; p < S->n_polys; ++p)
        for (int64_t s = S->poly_start[p]; s < S->poly_start[p + 1]; ++s) mono_poly[(size_t)s] = p;
    int64_t total = 0;
    for (int64_t s = 0; s < M; ++s) {
        if (total > 0x7FFFFFFF) return fail(PE_EUNSUPPORTED, "too many prescaled coefficients");
        start[(size_t)s] = (int32_t)total;
        const dd re{coef[4 * s + 0], coef[4 * s + 1]}, im{coef[4 * s + 2], coef[4 * s + 3]};
        for (int64_t j = S->mono_start[s]; j < S->mono_start[s + 1]; ++j) {
            const double a = (double)S->exp[(size_t)j];
            const dd r = dw_mul_d(re, a), i = dw_mul_d(im, a);
            pc.insert(pc.end(), {r.hi, r.lo, i.hi, i.lo});
        }
        pc.insert(pc.end(), {re.hi, re.lo, im.hi, im.lo});
        total += S->mono_start[s + 1] - S->mono_start[s] + 1;
    }
    if ((e = S->ab_mono_poly.upload(mono_poly.data(), mono_poly.size() * sizeof(int32_t))) !=
            hipSuccess ||
        (e = S->ab_pcoef_start.upload(start.data(), start.size() * sizeof(int32_t))) != hipSuccess ||
        (e = S->ab_pcoef.upload(pc.data(), pc.size() * sizeof(double))) != hipSuccess)
        return hip_fail(e, "uploading the prescaled coefficients");
    return PE_OK;
}

}  // namespace

extern "C" pe_status pe_eval_jac_paper_layout(pe_system sys, int64_t n_points, pe_cvec points,
                                              pe_cvec out_f, pe_cvec out_J,
                                              pe_precision precision, void *stream)
{
    if (!sys) return fail(PE_EINVAL, "NULL system");
    System *S = reinterpret_cast<System *>(sys);
    if (n_points < 0) return fail(PE_EINVAL, "n_points < 0");
    if (precision != PE_DD && precision != PE_FP64) return fail(PE_EINVAL, "unknown precision");
    if (n_points == 0) return PE_OK;
    const bool dd_mode = precision == PE_DD;
    if (!points.re_hi || !points.im_hi || !out_f.re_hi || !out_f.im_hi ||
        (dd_mode && (!points.re_lo || !points.im_lo || !out_f.re_lo || !out_f.im_lo)))
        return fail(PE_EINVAL, "a required plane is NULL");
    const bool jac = out_J.re_hi || out_J.re_lo || out_J.im_hi || out_J.im_lo;
    if (jac && (!out_J.re_hi || !out_J.im_hi || (dd_mode && (!out_J.re_lo || !out_J.im_lo))))
        return fail(PE_EINVAL, "out_J is partially NULL");
    if (S->max_k > 32) return fail(PE_EUNSUPPORTED, "monomials of more than 32 variables");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != S->device)
        return fail(PE_EINVAL, "the current device is not the system's device");

    std::lock_guard<std::mutex> lock(S->mu);
    pe_status st = upload_tables(S);
    if (st != PE_OK) return st;
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    const int words = dd_mode ? 4 : 2;
    const size_t units = (size_t)n_points * S->n_monos;
    const size_t mons_bytes = units * (S->n_vars + 1) * words * sizeof(double);
    hipError_t e = hipSuccess;
    if (S->ab_cf.bytes < units * words * sizeof(double) || S->ab_mons.bytes < mons_bytes ||
        S->ab_points != n_points || S->ab_words != words) {
        // the dense array's zeros depend on the layout: clear it when it changes
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(hs, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
            return fail(PE_EUNSUPPORTED,
                        "scratch must be laid out during stream capture: call once before capturing");
        (void)hipStreamSynchronize(hs);
        if (S->ab_cf.bytes < units * words * sizeof(double) &&
            (e = S->ab_cf.alloc(units * words * sizeof(double))) != hipSuccess)
            return hip_fail(e, "allocating common factors");
        if (S->ab_mons.bytes < mons_bytes && (e = S->ab_mons.alloc(mons_bytes)) != hipSuccess)
            return hip_fail(e, "allocating the dense term array");
        if (mons_bytes && (e = hipMemset(S->ab_mons.ptr, 0, mons_bytes)) != hipSuccess)
            return hip_fail(e, "clearing the dense term array");
        S->ab_points = n_points;
        S->ab_words = words;
    }
    AblationArgs a{};
    a.n_vars = S->n_vars;
    a.n_polys = S->n_polys;
    a.n_monos = S->n_monos;
    a.n_points = n_points;
    a.poly_start = (const int64_t *)S->d_poly_start.ptr;
    a.mono_start = (const int32_t *)S->d_mono_start.ptr;
    a.word = (const uint32_t *)S->d_word.ptr;
    a.mono_poly = (const int32_t *)S->ab_mono_poly.ptr;
    a.pcoef = (const double *)S->ab_pcoef.ptr;
    a.pcoef_start = (const int32_t *)S->ab_pcoef_start.ptr;
    const double *xp[4] = {points.re_hi, points.re_lo, points.im_hi, points.im_lo};
    double *fp[4] = {out_f.re_hi, out_f.re_lo, out_f.im_hi, out_f.im_lo};
    double *Jp[4] = {out_J.re_hi, out_J.re_lo, out_J.im_hi, out_J.im_lo};
    for (int q = 0; q < 4; ++q) {
        a.x[q] = xp[q];
        a.f[q] = fp[q];
        a.J[q] = jac ? Jp[q] : nullptr;
    }
    a.cf = (double *)S->ab_cf.ptr;
    a.mons = (double *)S->ab_mons.ptr;
    e = launch_ablation(dd_mode ? 1 : 0, a, S->max_k, hs);
    if (e != hipSuccess) return hip_fail(e, "launching the three-kernel evaluation");
    return PE_OK;
}
