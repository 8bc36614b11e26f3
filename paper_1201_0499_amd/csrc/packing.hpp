// Encodings shared by the host packer and the kernels (no HIP dependency).
#pragma once

#include <stdint.h>

namespace pe {

// One packed variable of a monomial: variable index in the low 24 bits,
// exponent minus one in the high 8 bits (the paper stores exponents minus
// one as well, Section 3.1).  Padding entries name the dummy variable n_vars,
// whose power-table column holds the value 1.
constexpr uint32_t kPosMask = 0x00FFFFFFu;
constexpr int kExpShift = 24;
// Runs are added in blocks of at most kRunBlock terms with the cascaded
// accumulator (whose error bound grows with the square of the number of
// terms), and the block sums are added with the sloppy sum.
constexpr int kRunBlock = 32;

inline uint32_t pack_word(int32_t pos, int32_t exp)
{
    return (uint32_t)pos | ((uint32_t)(exp - 1) << kExpShift);
}

}  // namespace pe
