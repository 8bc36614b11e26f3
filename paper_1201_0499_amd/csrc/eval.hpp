// Launch arguments shared by the host packer and the evaluation kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "packing.hpp"

namespace pe {

// LDS of one CDNA4 compute unit, the most one workgroup can take.
constexpr int kMaxLds = 160 * 1024;

// Mask entry of a point the evaluation computes (the Newton corrector's
// status of a start that is still running).
constexpr int32_t kMaskLive = -1;

struct EvalArgs {
    // system shape
    int32_t n_vars;
    int32_t n_polys;
    int32_t R;            // power-table rows: x^1 .. x^R
    int32_t L;            // lanes per monomial (power of two, <= 64)
    int32_t log2L;
    int32_t log2VG;       // monomials per staged value term = 2^log2VG
    int32_t log2S;        // lanes per output run in the summation = 2^log2S
    int32_t KP;           // padded variables per monomial = CC * L
    int32_t G;            // workgroups per polynomial and point
    int32_t stage_slots;  // LDS staging slots per chunk (last one is the discard slot)
    int32_t max_rows;     // longest run of any chunk (rows of the row table in LDS)
    int32_t n_groups;     // n_polys * G
    int32_t any_fold;     // 1 if some polynomial's constant last monomial is folded
    int32_t T;            // points per workgroup tile (1..32)
    int32_t nbuf;         // staging buffers: 1, or 2 (one barrier per item)
    // packed tables (schedule order = system order)
    const uint32_t *word;          // [M][KP]
    const uint16_t *dest;          // [M][KP] staging slot of each derivative term
    const uint16_t *vdest;         // [M] staging slot of each monomial's value
    const double *coef;            // [M][4]  re_hi, re_lo, im_hi, im_lo
    const int4 *chunk_info;        // [n_chunks]: first monomial, monomials | rows
                                   //   << 16, first row_start entry, chunk index
    const uint32_t *run_info;      // [n_chunks][n_vars+1]: output | run length << 16
                                   //   by rank (longest run first)
    const uint16_t *row_start;     // per chunk rows+1: first slot of each row
    const int4 *group_info;        // [n_groups][2]: first chunk, end chunk, then the
                                   //   first chunk's header (as in chunk_info)
    // points and outputs: four planes each
    int64_t n_points;
    const double *x[8];            // 4 planes (dd, FP64), 8 (quad-double)
    double *f[8];
    double *J[8];                  // J[0] == nullptr: no Jacobian
    const int32_t *mask;           // [n_points] or nullptr: skip points whose entry is not kMaskLive
    // cross-workgroup combination (G > 1)
    double *partial;               // [n_points][G][n_vars+1][n_polys][words]
};

// One system of a batch: its launch arguments (point and output pointers
// unset) and the element offsets of its points, values and Jacobians in the
// batch's concatenated buffers.
struct BatchDesc {
    EvalArgs a;
    int64_t x_off, f_off, J_off;
};

// One task of the persistent batch kernel: point pt of system sys,
// polynomials p0 .. p1-1.
struct BatchTask {
    int32_t sys, p0, p1, pad;
    int64_t pt;
};

struct BatchArgs {
    const BatchDesc *desc;
    const BatchTask *tasks;
    int64_t n_tasks;
    const double *x[4];
    double *f[4];
    double *J[4];
};

hipError_t launch_batch(int prec, int cc, int maxt, const BatchArgs &args, dim3 grid, dim3 block,
                        size_t lds_bytes, hipStream_t stream);

// Workgroups of the batch kernel resident per compute unit (at least 1).
int batch_occupancy(int prec, int cc, int maxt, int threads, size_t lds_bytes);

// Launch one evaluation.  prec: 0 = FP64, 1 = double-double, 2 =
// quad-double (256 threads, chunk_vars 2 or 4 only).
hipError_t launch_eval(int prec, int cc, int maxt, const EvalArgs &args, dim3 grid, dim3 block,
                       size_t lds_bytes, hipStream_t stream);

// After an evaluation with G > 1: add the partial rows into f and J
// (prec as for launch_eval).
hipError_t launch_combine(int prec, const EvalArgs &args, hipStream_t stream);

// Raise the dynamic LDS limit of every kernel instantiation (call once).
hipError_t eval_kernels_init();

// Size of the library's static device scratch, the buffer of the partial
// rows of the cross-workgroup combination in pe_eval_jac_noalloc.  Every
// device the library runs on holds one such array until the process ends.
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;

// Looks up the address of the static scratch on the current device and
// keeps it; call with the device current, once per device, at set-up.
hipError_t static_scratch_setup();

// The address kept by static_scratch_setup for `device` (nullptr if that
// device was never set up).  Reads only: no HIP call, no allocation.
void *static_scratch_ptr(int device);

}  // namespace pe
