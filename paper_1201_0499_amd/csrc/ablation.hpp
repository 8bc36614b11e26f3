// The paper's three-kernel evaluation (definitions and description in
// ablation.hip), for comparison with the fused kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pe {

struct AblationArgs {
    int32_t n_vars, n_polys;
    int64_t n_monos, n_points;
    const int64_t *poly_start;   // [n_polys+1]
    const int32_t *mono_start;   // [M+1] into word
    const uint32_t *word;        // packed (variable, exponent-1)
    const int32_t *mono_poly;    // [M] polynomial of each monomial
    const double *pcoef;         // prescaled coefficients, 4 words each
    const int32_t *pcoef_start;  // [M] first prescaled coefficient of a monomial (k + 1 each)
    const double *x[4];          // points [P][n]
    double *f[4];                // values [P][n_polys]
    double *J[4];                // Jacobians [P][n][n_polys]; J[0] == nullptr: none
    double *cf;                  // common factors, planes [words][P*M]
    double *mons;                // dense terms: per point and polynomial, n+1 rows of m entries
};

// The three kernels in order on `stream`; prec 0 FP64, 1 double-double;
// kmax >= the largest monomial size (at most 32).
hipError_t launch_ablation(int prec, const AblationArgs &a, int kmax, hipStream_t stream);

}  // namespace pe
