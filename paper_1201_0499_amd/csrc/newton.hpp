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
    double *x[4];
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
    const double *x[4];            // dd points [P][n]
    double *f[4];                  // dd values [P][n_polys]
    const int32_t *status;         // [P] or nullptr: only kRunning points are evaluated
};

// f(x) in complex double-double, values only (one workgroup per point).
// Raise the dynamic LDS limit of the residual kernel (once per process).
hipError_t newton_kernels_init();

hipError_t launch_resid(const ResidArgs &a, hipStream_t stream);

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

// x <- x - d for running starts (x in dd; d in FP64 when prec == 0, else dd),
// iters += 1.
hipError_t launch_update(int prec, int64_t n_starts, int32_t n, double *const x[4],
                         const double *const d[4], const int32_t *status, int32_t *iters,
                         hipStream_t stream);

// status = kRunning, iters = 0 for every start.
hipError_t launch_newton_init(int64_t n_starts, int32_t *status, int32_t *iters, hipStream_t stream);

}  // namespace pe
