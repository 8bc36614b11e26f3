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
// Piece table entry: output index in the low 21 bits; for the first piece of
// an output within a chunk, the number of pieces of that output in the high
// 11 bits (0 for the other pieces).  Pieces of one output are consecutive
// (their sums land in consecutive staging slots) and all but the last hold
// exactly PL terms.
constexpr uint32_t kOutMask = 0x001FFFFFu;
constexpr int kRunShift = 21;
constexpr int kMaxRun = 2047;
// Longest piece: a piece is added with the cascaded accumulator, whose error
// bound grows with the square of the number of terms.
constexpr int kMaxPiece = 32;

inline uint32_t pack_word(int32_t pos, int32_t exp)
{
    return (uint32_t)pos | ((uint32_t)(exp - 1) << kExpShift);
}

}  // namespace pe
