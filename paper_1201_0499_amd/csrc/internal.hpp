// Host-side objects behind the opaque handles of polyeval.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <mutex>
#include <vector>

#include "polyeval.h"
#include "eval.hpp"

namespace pe {

pe_status fail(pe_status st, const char *fmt, ...);
int ilog2(int v);
int next_pow2(int v);
pe_status hip_fail(hipError_t e, const char *what);
hipError_t library_init();

// Owned device allocation.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf();
    hipError_t alloc(size_t n);
    hipError_t upload(const void *src, size_t n);
};

// Packed tables of one system for one launch schedule.
struct Schedule {
    int L = 1, cc = 4, nt = 256, G = 1;  // key
    int KP = 0, MC = 0, R = 1, n_vars = 0, VG = 1;
    int stage_slots = 1, n_chunks = 0, max_rows = 0;
    int any_fold = 0;  // some group starts its value output at a folded constant
    DevBuf word, dest, vdest;
    DevBuf chunk_info, run_info, row_start, group_info;
    // LDS of one workgroup: T power tables and accumulator rows, nbuf
    // staging areas and row tables
    size_t lds_bytes(int words, int T = 1, int nbuf = 1) const;
};

struct System {
    int32_t n_vars = 0, n_polys = 0;
    int64_t n_monos = 0;
    int max_k = 0, max_exp = 1;
    int device = 0;
    std::vector<int64_t> poly_start, mono_start;
    std::vector<int32_t> pos, exp;
    DevBuf coef;  // [M][4]
    // schedule selection: pinned values (0 = automatic)
    int pin_L = 0, pin_cc = 0, pin_nt = 0, pin_G = 0;
    // points per tile and staging buffers (0 = automatic)
    int pin_T = 0, pin_nbuf = 0;
    std::vector<std::unique_ptr<Schedule>> schedules;
    // partial rows of the cross-workgroup combination
    DevBuf partial;
    // CSR tables of the values-only residual kernel
    DevBuf d_poly_start, d_mono_start, d_word;
    // Newton workspace (grown on demand)
    DevBuf nw_J, nw_r, nw_d, nw_f64, nw_counter;
    // path tracker: total degrees of the polynomials (uploaded once),
    // accepted points and per-path state
    DevBuf tk_deg, tk_xs, tk_state;
    // the paper's three-kernel evaluation: monomial -> polynomial, prescaled
    // coefficients, common factors, dense term array (and its layout)
    DevBuf ab_mono_poly, ab_pcoef, ab_pcoef_start, ab_cf, ab_mons;
    int64_t ab_points = -1;
    int ab_words = 0;
    std::mutex mu;

    // the schedule key for n_points: the pinned one, else the automatic one
    void schedule_key(int64_t n_points, int &L, int &cc, int &nt, int &G) const;
    pe_status schedule_for(int64_t n_points, Schedule **out);
    // the schedule for n_points only if its tables exist (builds nothing)
    pe_status find_schedule(int64_t n_points, Schedule **out) const;
    // points per tile and staging buffers of a launch of schedule sc over
    // n_points points: the pinned values, else the automatic ones; 0 when
    // the pinned ones do not fit the LDS
    void launch_shape(const Schedule &sc, int64_t n_points, bool dd, int &T, int &nbuf) const;
    pe_status schedule_with(int L, int cc, int nt, int G, Schedule **out);
    // launch arguments of a schedule (points, outputs and mask unset)
    void fill_args(const Schedule &sc, EvalArgs &a) const;
    // evaluation with the lock held; J[0] == nullptr skips the Jacobian,
    // mask (optional) skips points whose entry is not -1.  no_alloc: use
    // only existing schedule tables and the static scratch, allocate nothing
    pe_status eval_locked(int64_t n_points, const double *const x[4], double *const f[4],
                          double *const J[4], bool dd, hipStream_t stream, const int32_t *mask,
                          bool no_alloc = false);
};

// Newton's method from n_starts starts (the body of pe_newton, called with
// the system's lock held).  init: set every start running first; else only
// the starts whose status is kRunning iterate and iters_out must be zero
// for them.
pe_status newton_run(System *S, int64_t n_starts, pe_cvec x, double tol, int32_t max_iter,
                     bool mixed, double *res_out, int32_t *iters_out, int32_t *status_out,
                     hipStream_t hs, bool init);

}  // namespace pe
