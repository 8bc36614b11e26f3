// Host-side packing of a system for one launch schedule (pure C++, no HIP).
//
// The summation of Section 3.3 is done without the paper's zero-padded term
// array: within a chunk of monomials, every derivative term gets an LDS
// staging slot such that the terms of one output are contiguous and ordered
// by monomial; the monomial values are first summed inside each wave and
// take one slot per wave, after all derivative terms.  The run of each output is cut into pieces of at
// most PL terms; a lane sums one piece (the sum is stored in place of the
// piece's first term) and the first piece of every output then adds the
// pieces of its output into the accumulator.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace pe {

struct CsrView {
    int32_t n_vars, n_polys;
    int64_t n_monos;
    const int64_t *poly_start;
    const int64_t *mono_start;
    const int32_t *pos;
    const int32_t *exp;
};

struct ScheduleTables {
    int L = 1, cc = 4, nt = 256, G = 1;
    int KP = 0, MC = 0;
    int stage_slots = 1;  // max terms per chunk + 1 discard slot
    int n_chunks = 0;
    int max_pieces = 0;
    std::vector<uint32_t> word;         // [M][KP]
    std::vector<uint16_t> dest;         // [M][KP]
    std::vector<int32_t> chunk_info;    // [n_chunks][4]: first monomial,
                                        //   monomials | first value slot << 16,
                                        //   first piece, n_pieces | PL << 16
    std::vector<uint16_t> piece_start;  // per chunk n_pieces+1 entries
    std::vector<uint32_t> piece_out;    // per chunk n_pieces entries (packing.hpp)
    std::vector<int32_t> group_chunk0;  // [n_polys*G+1]
    std::vector<int32_t> group_info;    // [n_polys*G][8]: first chunk, end chunk,
                                        //   then the first chunk's 4 header ints
};

// Fill `t` for the schedule (t.L, t.cc, t.nt, t.G).  Returns an empty string
// on success, else a message.
std::string build_schedule_tables(const CsrView &S, ScheduleTables &t);

}  // namespace pe
