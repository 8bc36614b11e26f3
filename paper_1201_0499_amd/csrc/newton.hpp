// Kernels of the Newton corrector (launch wrappers; definitions in
// newton.hip).  Per start the corrector keeps a status word:
//   kRunning (-1) while iterating, then 0 converged, 1 iteration limit,
//   2 zero pivot (singular Jacobian), 3 non-finite residual.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pe {

constexpr int32_t kRunning = -1;

struct LuPlanes {
    double *J[4];
    const double *r[4];
    double *d[4];
};

struct UpdPlanes {
    double *x[8];
    const double *d[4];
};

struct ResidArgs {
    int32_t n_vars, n_polys;
    int32_t R;                     // power rows x^1 .. x^R, R = maximal exponent
    const int64_t *poly_start;     // [n_polys+1]
    const int32_t *mono_start;     // [M+1] into word
    const uint32_t *word;          // [nnz] packed (variable, exponent-1)
    const double *coef;            // [M][4]
    int64_t n_points;
    const double *x[8];            // points [P][n]: dd planes 0..3, or quad-double 0..7
    double *f[8];                  // values [P][n_polys], planes as x
    const int32_t *status;         // [P] or nullptr: only kRunning points are evaluated
};

// Raise the dynamic LDS limit of the residual kernels (once per process).
hipError_t newton_kernels_init();

// f(x), values only (one workgroup per point), in complex double-double
// (prec 1, planes re hi, re lo, im hi, im lo) or complex quad-double (prec 2,
// planes re x0..x3, im x0..x3).  resid_fits: the power table x^1 .. x^R of
// n variables fits in LDS.
hipError_t launch_resid(const ResidArgs &a, int prec, hipStream_t stream);
bool resid_fits(int prec, int32_t n, int32_t R);

// Per start: res = max_p |f_p| (from the leading words); update status:
// non-finite -> 3, res < tol -> 0, iters >= max_iter -> 1; count the starts
// still running into *running (which the caller zeroes).
hipError_t launch_check(int64_t n_starts, int32_t n_polys, const double *const f[4], double tol,
                        int32_t max_iter, double *res, const int32_t *iters, int32_t *status,
                        int32_t *running, hipStream_t stream);

// Solve J d = r per running start by blocked Gaussian elimination with
// partial pivoting: J column-major [S][n][n] (overwritten), rhs r [S][n],
// solution d [S][n].  prec 0: complex FP64 (re_hi/im_hi planes), 1: complex
// dd.  A zero or non-finite pivot sets status 2.  The factored panel lives
// in LDS: lu_solve_fits(prec, n) tells whether n is small enough.
hipError_t launch_lu_solve(int prec, int64_t n_starts, int32_t n, double *const J[4],
                           const double *const r[4], double *const d[4], int32_t *status,
                           hipStream_t stream);

bool lu_solve_fits(int prec, int32_t n);

// x <- x - d for running starts, iters += 1: prec 0, x in dd (4 planes) and
// d in FP64 (planes 0 and 2); prec 1, both in dd; prec 2, x in quad-double
// (8 planes) and d in FP64.
hipError_t launch_update(int prec, int64_t n_starts, int32_t n, double *const *x,
                         const double *const d[4], const int32_t *status, int32_t *iters,
                         hipStream_t stream);

// status = kRunning, iters = 0 for every start.
hipError_t launch_newton_init(int64_t n_starts, int32_t *status, int32_t *iters, hipStream_t stream);

}  // namespace pe
