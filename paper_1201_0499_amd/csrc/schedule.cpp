// Host-side packing of a system for one launch schedule.  See schedule.hpp.
#include "schedule.hpp"

#include <algorithm>

#include "packing.hpp"

namespace pe {

std::string build_schedule_tables(const CsrView &S, ScheduleTables &t)
{
    const int KP = t.cc * t.L;
    const int MC = t.nt / t.L;
    if (KP < 1 || MC < 1 || t.G < 1) return "invalid schedule";
    if (S.n_vars >= (int32_t)kOutMask) return "too many variables for the piece encoding";
    t.KP = KP;
    t.MC = MC;
    {
        // value terms per chunk about the length of a derivative output's run
        const double kbar = S.n_monos > 0 ? (double)(S.mono_start[S.n_monos] - S.mono_start[0]) /
                                                (double)S.n_monos
                                          : 1.0;
        const double want = (double)S.n_vars / std::max(1.0, kbar);
        int vg = 1;
        while (2 * vg <= want + 0.5 && 2 * vg * t.L <= 64) vg *= 2;
        t.VG = vg;
    }
    const int VG = t.VG;
    const int64_t M = S.n_monos;
    const int n = S.n_vars;
    t.word.assign((size_t)M * KP, (uint32_t)n);
    t.dest.assign((size_t)M * KP, 0);
    t.vdest.assign((size_t)M, 0);
    t.chunk_info.clear();
    t.piece_len.clear();
    t.piece_out.clear();
    t.group_chunk0.clear();
    int stage_slots = 1;
    int max_pieces = 0;

    struct Term {
        int32_t out;
        int32_t seq;  // monomial * KP + variable: monomial order within an output
    };
    std::vector<Term> terms;
    std::vector<int32_t> runs;
    std::vector<int32_t> slot;

    for (int p = 0; p < S.n_polys; ++p) {
        const int64_t s0 = S.poly_start[p], s1 = S.poly_start[p + 1];
        const int64_t nm = s1 - s0;
        const int nch = (int)((nm + MC - 1) / MC);
        const int first_chunk = (int)(t.chunk_info.size() / 4);
        for (int c = 0; c < nch; ++c) {
            const int64_t a = s0 + (int64_t)c * MC;
            const int64_t b = std::min<int64_t>(s1, a + MC);
            terms.clear();
            for (int64_t s = a; s < b; ++s) {
                const int sl = (int)(s - a);
                const int64_t e0 = S.mono_start[s], e1 = S.mono_start[s + 1];
                const int k = (int)(e1 - e0);
                if (k > KP) return "a monomial has more variables than lanes*chunk_vars";
                for (int j = 0; j < k; ++j) {
                    t.word[(size_t)s * KP + j] = pack_word(S.pos[e0 + j], S.exp[e0 + j]);
                    terms.push_back({S.pos[e0 + j], sl * KP + j});
                }
                if (sl % VG == 0) terms.push_back({n, sl * KP});  // value of sl .. sl+VG-1
            }
            std::sort(terms.begin(), terms.end(), [](const Term &x, const Term &y) {
                return x.out != y.out ? x.out < y.out : x.seq < y.seq;
            });
            const int T = (int)terms.size();
            runs.clear();
            int max_run = 0;
            for (int r = 0; r < T;) {
                int e = r + 1;
                while (e < T && terms[e].out == terms[r].out) ++e;
                runs.push_back(e - r);
                max_run = std::max(max_run, e - r);
                r = e;
            }
            // piece length: minimize the summation's critical path, i.e. the
            // rounds of pieces per lane times PL terms (8 instructions per
            // term in a piece) plus the longest run of pieces (11 per piece
            // sum), among the lengths whose staging table fits
            int PL = 0, best = -1, NP = 0;
            for (int cand = 1; cand <= std::min(max_run, kMaxPiece); ++cand) {
                int np = 0, worst_run = 0;
                for (int len : runs) {
                    const int r = (len + cand - 1) / cand;
                    np += r;
                    worst_run = std::max(worst_run, r);
                }
                if (worst_run > kMaxRun || np > 65535) continue;
                const int64_t slots = (int64_t)cand * np;
                if (slots + 1 > 65535) continue;
                if (t.max_stage > 0 && slots + 1 > t.max_stage) continue;
                const int cost = 8 * ((np + t.nt - 1) / t.nt) * cand + 11 * worst_run;
                if (best < 0 || cost < best) {
                    best = cost;
                    PL = cand;
                    NP = np;
                }
            }
            if (PL == 0) return "the term staging of a chunk does not fit (too many terms)";
            // slots: term i of piece l at i*NP + l
            slot.assign((size_t)T, 0);
            int r0 = 0, l = 0;
            const int piece0 = (int)t.piece_out.size();
            for (int len : runs) {
                const int out = terms[r0].out;
                const int nrun = (len + PL - 1) / PL;
                for (int off = 0; off < len; off += PL, ++l) {
                    const int plen = std::min(PL, len - off);
                    for (int i = 0; i < plen; ++i) slot[(size_t)(r0 + off + i)] = i * NP + l;
                    t.piece_len.push_back((uint16_t)plen);
                    t.piece_out.push_back((uint32_t)out |
                                          (off == 0 ? (uint32_t)nrun << kRunShift : 0u));
                }
                r0 += len;
            }
            for (int r = 0; r < T; ++r) {
                const int sl = terms[r].seq / KP;
                const int j = terms[r].seq % KP;
                if (terms[r].out == n)
                    t.vdest[(size_t)(a + sl)] = (uint16_t)slot[(size_t)r];
                else
                    t.dest[(size_t)(a + sl) * KP + j] = (uint16_t)slot[(size_t)r];
            }
            stage_slots = std::max(stage_slots, PL * NP + 1);
            const int npieces = NP;
            t.chunk_info.push_back((int32_t)a);
            t.chunk_info.push_back((int32_t)(b - a));
            t.chunk_info.push_back(piece0);
            t.chunk_info.push_back(npieces | (PL << 16));
            max_pieces = std::max(max_pieces, npieces);
        }
        for (int g = 0; g < t.G; ++g)
            t.group_chunk0.push_back(first_chunk + (int)(((int64_t)nch * g) / t.G));
    }
    t.group_chunk0.push_back((int)(t.chunk_info.size() / 4));
    const size_t n_groups = t.group_chunk0.size() - 1;
    t.group_info.assign(n_groups * 8, 0);
    for (size_t g = 0; g < n_groups; ++g) {
        const int c0 = t.group_chunk0[g], c1 = t.group_chunk0[g + 1];
        t.group_info[8 * g + 0] = c0;
        t.group_info[8 * g + 1] = c1;
        if (c0 < c1)
            for (int j = 0; j < 4; ++j) t.group_info[8 * g + 2 + j] = t.chunk_info[4 * (size_t)c0 + j];
    }
    t.stage_slots = stage_slots;
    t.n_chunks = (int)(t.chunk_info.size() / 4);
    t.max_pieces = max_pieces;
    const uint16_t trash = (uint16_t)(stage_slots - 1);
    for (int64_t s = 0; s < M; ++s) {
        const int k = (int)(S.mono_start[s + 1] - S.mono_start[s]);
        for (int j = k; j < KP; ++j) t.dest[(size_t)s * KP + j] = trash;
    }
    return std::string();
}

}  // namespace pe
