// Host-side packing of a system for one launch schedule.  See schedule.hpp.
#include "schedule.hpp"

#include <algorithm>
#include <climits>

#include "packing.hpp"

namespace pe {

std::string build_schedule_tables(const CsrView &S, ScheduleTables &t)
{
    const int KP = t.cc * t.L;
    const int MC = t.nt / t.L;
    if (KP < 1 || MC < 1 || t.G < 1) return "invalid schedule";
    if (S.n_vars + 1 > 65535) return "too many variables for the run tables";
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
    t.run_info.clear();
    t.row_start.clear();
    t.group_chunk0.clear();
    t.any_fold = 0;
    int stage_slots = 1, max_rows = 0;
    std::vector<int32_t> len_of, order, rank_of;

    struct Term {
        int32_t out;
        int32_t seq;  // monomial * KP + variable: monomial order within an output
    };
    std::vector<Term> terms;

    std::vector<int32_t> folded((size_t)S.n_polys, 0);
    for (int p = 0; p < S.n_polys; ++p) {
        const int64_t s0 = S.poly_start[p];
        int64_t s1 = S.poly_start[p + 1];
        // a constant last monomial needs no lanes: its coefficient starts
        // the value output's accumulator instead of taking a chunk's slot
        if (s1 > s0 && S.mono_start[s1] == S.mono_start[s1 - 1]) {
            if (s1 - 1 >= (int64_t)INT32_MAX) return "too many monomials";
            folded[(size_t)p] = (int32_t)s1;  // monomial index + 1
            t.any_fold = 1;
            --s1;
        }
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
            if (T + 1 > 65535) return "too many terms in one chunk";
            if (t.max_stage > 0 && T + 1 > t.max_stage)
                return "the term staging of a chunk does not fit (too many terms)";
            // outputs by run length, longest first (ties by output); row i
            // holds the i-th term (in monomial order) of every output whose
            // run is longer than i, the j-th longest output at row_start[i] + j
            len_of.assign((size_t)n + 1, 0);
            for (const Term &x : terms) ++len_of[(size_t)x.out];
            order.resize((size_t)n + 1);
            for (int o = 0; o <= n; ++o) order[(size_t)o] = o;
            std::stable_sort(order.begin(), order.end(),
                             [&](int x, int y) { return len_of[(size_t)x] > len_of[(size_t)y]; });
            rank_of.assign((size_t)n + 1, 0);
            for (int j = 0; j <= n; ++j) {
                rank_of[(size_t)order[(size_t)j]] = j;
                t.run_info.push_back((uint32_t)order[(size_t)j] |
                                     ((uint32_t)len_of[(size_t)order[(size_t)j]] << 16));
            }
            const int rows = len_of[(size_t)order[0]];
            const int row0 = (int)t.row_start.size();
            int acc_rows = 0;
            for (int i = 0; i < rows; ++i) {
                t.row_start.push_back((uint16_t)acc_rows);
                int cnt = 0;
                while (cnt <= n && len_of[(size_t)order[(size_t)cnt]] > i) ++cnt;
                acc_rows += cnt;
            }
            t.row_start.push_back((uint16_t)acc_rows);  // == T
            max_rows = std::max(max_rows, rows);
            // terms are sorted by (output, monomial): the i-th term of each
            // output is the i-th of its run
            for (int q = 0; q < T;) {
                const int o = terms[q].out;
                int i = 0;
                for (; q < T && terms[q].out == o; ++q, ++i) {
                    const int slot = t.row_start[(size_t)row0 + i] + rank_of[(size_t)o];
                    const int sl = terms[q].seq / KP;
                    const int j = terms[q].seq % KP;
                    if (o == n)
                        t.vdest[(size_t)(a + sl)] = (uint16_t)slot;
                    else
                        t.dest[(size_t)(a + sl) * KP + j] = (uint16_t)slot;
                }
            }
            stage_slots = std::max(stage_slots, T + 1);
            const int32_t chunk = (int32_t)(t.chunk_info.size() / 4);
            t.chunk_info.push_back((int32_t)a);
            t.chunk_info.push_back((int32_t)(b - a) | (rows << 16));
            t.chunk_info.push_back(row0);
            t.chunk_info.push_back(chunk);
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
        // the folded constant goes to the polynomial's first group only
        if (g % (size_t)t.G == 0) t.group_info[8 * g + 6] = folded[g / (size_t)t.G];
    }
    t.stage_slots = stage_slots;
    t.max_rows = max_rows;
    t.n_chunks = (int)(t.chunk_info.size() / 4);
    const uint16_t trash = (uint16_t)(stage_slots - 1);
    for (int64_t s = 0; s < M; ++s) {
        const int k = (int)(S.mono_start[s + 1] - S.mono_start[s]);
        for (int j = k; j < KP; ++j) t.dest[(size_t)s * KP + j] = trash;
    }
    return std::string();
}

}  // namespace pe
