// Kernels of the path tracker (definitions in track.hip).
//
// Total-degree homotopy H(x, t) = (1 - t) * gamma * G(x) + t * F(x) with the
// start system G_i(x) = x_i^{d_i} - 1, d_i the total degree of f_i, tracked
// from t = 0 to t = 1 in complex FP64 by an Euler predictor along the
// tangent dx/dt = -H_x^{-1} H_t and a Newton corrector at the predicted t,
// with step-size control.  Paths run in lockstep: every round evaluates F
// and its Jacobian at each running path's current x (one masked launch of
// the evaluator), forms the homotopy's Jacobian and right-hand side for the
// path's phase, solves (the batched elimination), and applies the phase's
// update.  Finding roots of polynomial systems by continuation is the use
// the paper's introduction names for fast evaluation (Section 1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pe {

// Per-path status values of the tracker beyond the Newton ones (0 done,
// 2 zero pivot, 3 non-finite, kRunning while tracking).
constexpr int32_t kTrackStepUnderflow = 1;
constexpr int32_t kTrackStepLimit = 4;
constexpr int32_t kTrackEndgameFailed = 5;

struct TrackArgs {
    int64_t n_paths;
    int32_t n;
    double gamma_re, gamma_im;
    const int32_t *deg;    // [n] total degree of f_i (>= 1)
    double h_min, h_max;   // step bounds in t
    double corr_tol;       // accept when max|dx| <= corr_tol * (1 + max|x|)
    int32_t corr_iters;    // Newton iterations per corrector
    int32_t max_steps;     // step attempts per path
    double *x[2];          // current x, FP64 planes (re, im) [P][n]
    const double *f[2];    // F(x) [P][n]
    double *J[2];          // J_F on entry to the homotopy kernel, H_x after; column-major [P][n][n]
    double *r[2];          // right-hand side [P][n]
    const double *d[2];    // solution of H_x d = r [P][n]
    double *xs[2];         // last accepted x [P][n]
    double *t;             // [P] accepted t
    double *t1;            // [P] t of the step under correction
    double *h;             // [P] step size
    int32_t *phase;        // [P] 0: predict next; c >= 1: corrector iteration c
    int32_t *succ;         // [P] consecutive accepted steps
    int32_t *steps;        // [P] step attempts
    int32_t *status;       // [P] kRunning while tracking
    int32_t *running;      // count of running paths after a round (zeroed by the caller)
};

// x planes (dd, [P][n]) <- start solutions first .. first+P-1 of G: path
// index q has mixed-radix digits k_i in base d_i (digit of variable 0
// fastest) and x_i = exp(2 pi i k_i / d_i); low words zero.
hipError_t launch_track_start(int64_t first, int64_t n_paths, int32_t n, const int32_t *deg,
                              double *const x[4], hipStream_t stream);

// Per running path: t = 0, h = h_init, phase 0, counters 0, xs = x, low
// words of x zeroed, status kRunning.
hipError_t launch_track_init(const TrackArgs &a, double h_init, double *const xlo[2],
                             hipStream_t stream);

// H_x and the right-hand side for the path's phase: predictor at (x, t):
// H_x v = H_t = F - gamma G; corrector at (x, t1): H_x d = H(x, t1).
hipError_t launch_track_homotopy(const TrackArgs &a, hipStream_t stream);

// The phase's update after the solve (one wave per path), then counts the
// paths still running into *running.
hipError_t launch_track_step(const TrackArgs &a, hipStream_t stream);

// Before the endgame: tracked[p] = (status[p] == 0), and those paths are
// set running again (for the Newton corrector at t = 1).
hipError_t launch_track_endgame(int64_t n_paths, int32_t *tracked, int32_t *status,
                                hipStream_t stream);

// After the endgame: a path that went into it and did not converge gets
// kTrackEndgameFailed.
hipError_t launch_track_end(int64_t n_paths, const int32_t *tracked, int32_t *status,
                            hipStream_t stream);

}  // namespace pe
