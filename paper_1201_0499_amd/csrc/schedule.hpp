// Host-side packing of a system for one launch schedule (pure C++, no HIP).
//
// The summation of Section 3.3 is done without the paper's zero-padded term
// array.  Within a chunk of monomials the terms are ordered by output, then
// by monomial: k derivative terms per monomial, and one value term per VG
// consecutive monomials (their values are first added inside the wave, so
// that the value output's run is about as long as a derivative output's:
// VG ~ n / mean k); the value output is the last.  The outputs of a chunk
// are ranked by the length of their runs, longest first; row i of the LDS
// staging area holds the i-th term of every output whose run is longer than
// i, the j-th ranked output's at slot row_start[i] + j.  In the kernel the
// lane(s) of rank j add output j's run reading slot row_start[i] + j for
// i = 0, 1, ...: at every step consecutive lanes read consecutive slots,
// free of LDS bank conflicts, and every output sums in monomial order (the
// paper's one thread per output, per chunk).  A constant monomial that comes
// last in its polynomial takes no chunk slot: its coefficient is the initial
// value of the polynomial's value output (in its first workgroup).
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
    int VG = 1;           // monomials per value term (power of two, <= 64 / L)
    int stage_slots = 1;  // max terms per chunk + 1 discard slot
    int max_rows = 0;     // longest run of a chunk
    int max_stage = 0;    // if > 0: chunks whose terms + 1 exceed it are refused
    int n_chunks = 0;
    int any_fold = 0;     // 1 if some polynomial's constant last monomial is folded
    std::vector<uint32_t> word;         // [M][KP]
    std::vector<uint16_t> dest;         // [M][KP] derivative terms' slots
    std::vector<uint16_t> vdest;        // [M] value term's slot (read for the first
                                        //   monomial of each group of VG)
    std::vector<int32_t> chunk_info;    // [n_chunks][4]: first monomial,
                                        //   monomials | rows << 16, first entry
                                        //   in row_start, chunk index
    std::vector<uint32_t> run_info;     // [n_chunks][n_vars+1]: rank j -> output
                                        //   | run length << 16 (value output n_vars)
    std::vector<uint16_t> row_start;    // per chunk rows+1 entries: first slot of
                                        //   each row, then the number of terms
    std::vector<int32_t> group_chunk0;  // [n_polys*G+1]
    std::vector<int32_t> group_info;    // [n_polys*G][8]: first chunk, end chunk,
                                        //   the first chunk's 4 header ints, then
                                        //   1 + the index of a folded constant
                                        //   monomial (0: none), and 0
};

// Fill `t` for the schedule (t.L, t.cc, t.nt, t.G).  Returns an empty string
// on success, else a message.
std::string build_schedule_tables(const CsrView &S, ScheduleTables &t);

}  // namespace pe
