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
    const int64_t M = S.n_monos;
    const int n = S.n_vars;
    t.word.assign((size_t)M * KP, (uint32_t)n);
    t.dest.assign((size_t)M * KP, 0);
    t.vdest.assign((size_t)M, 0);
    t.chunk_info.clear();
    t.piece_start.clear();
    t.piece_out.clear();
    t.group_chunk0.clear();
    int stage_slots = 1;
    int max_pieces = 0;

    struct Term {
        int32_t out;
        int32_t seq;
    };
    std::vector<Term> terms;
    std::vector<int32_t> runs;

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
                    terms.push_back({S.pos[e0 + j], sl * (KP + 1) + j});
                }
                terms.push_back({n, sl * (KP + 1) + KP});
            }
            std::sort(terms.begin(), terms.end(), [](const Term &x, const Term &y) {
                return x.out != y.out ? x.out < y.out : x.seq < y.seq;
            });
            const int T = (int)terms.size();
            if (T + 1 > 65535) return "too many terms in one chunk";
            for (int r = 0; r < T; ++r) {
                const int sl = terms[r].seq / (KP + 1);
                const int j = terms[r].seq % (KP + 1);
                const int64_t s = a + sl;
                if (j == KP)
                    t.vdest[(size_t)s] = (uint16_t)r;
                else
                    t.dest[(size_t)s * KP + j] = (uint16_t)r;
            }
            stage_slots = std::max(stage_slots, T + 1);
            runs.clear();
            int max_run = 0;
            for (int r = 0; r < T;) {
                int e = r + 1;
                while (e < T && terms[e].out == terms[r].out) ++e;
                runs.push_back(e - r);
                max_run = std::max(max_run, e - r);
                r = e;
            }
            // pieces: aim at one piece per lane; never fewer pieces than outputs
            const int cap = std::max<int>(t.nt, (int)runs.size());
            int PL = std::max(1, (T + t.nt - 1) / t.nt);
            for (;;) {
                int np = 0;
                for (int len : runs) np += (len + PL - 1) / PL;
                if (np <= cap || PL >= max_run) break;
                ++PL;
            }
            int r0 = 0, npieces = 0;
            const int piece0 = (int)t.piece_out.size();
            for (int len : runs) {
                const int out = terms[r0].out;
                const int nrun = (len + PL - 1) / PL;
                for (int off = 0; off < len; off += PL) {
                    t.piece_start.push_back((uint16_t)(r0 + off));
                    t.piece_out.push_back((uint32_t)out |
                                          (off == 0 ? (uint32_t)nrun << kRunShift : 0u));
                    ++npieces;
                }
                r0 += len;
            }
            t.piece_start.push_back((uint16_t)T);
            if (npieces > 65535 || PL > 65535) return "too many pieces in one chunk";
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
