// LDS sizing rules of the kernels that take a dynamic LDS area, shared by
// the launch code and the CPU tests (pure C++, no HIP dependency).
#pragma once

#include <stddef.h>

namespace pe {

// LDS of one CDNA4 compute unit, the most one workgroup can take.
constexpr size_t kLdsBytes = 160 * 1024;

// Bytes of static __shared__ arrays the blocked elimination kernel declares
// beside its dynamic panel (the first panel's multipliers of the second
// panel's top rows, NB x NB complex values: 4 KiB in FP64 and 2 KiB in
// double-double; per-wave pivot candidates, pivot rows, a permutation of up
// to 2 NB rows: under 0.5 KiB), rounded up.
constexpr size_t kLuStaticLds = 5 * 1024;

// Panel width of the blocked elimination: `widest` columns (16 in FP64, 8
// in double-double), halved while `width x n` complex values of `elem`
// bytes and the kernel's static arrays would exceed the LDS, down to 2;
// 0 if not even two columns fit.
inline int lu_panel_width(size_t elem, long n, int widest)
{
    for (int nb = widest; nb >= 2; nb >>= 1)
        if ((size_t)nb * (size_t)n * elem + kLuStaticLds <= kLdsBytes) return nb;
    return 0;
}

}  // namespace pe
