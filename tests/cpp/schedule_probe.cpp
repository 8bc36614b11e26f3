// Test-only shim: exposes the library's host packer (schedule.cpp) to the
// CPU tests through a small C interface.  Built with g++ by the tests.
#include <cstring>
#include <string>

#include "lds_budget.hpp"
#include "schedule.hpp"

using pe::ScheduleTables;

static int g_max_stage = 0;

extern "C" {

// panel width of the blocked elimination for n and `elem`-byte values
int probe_lu_panel(int elem, long n, int widest) { return pe::lu_panel_width((size_t)elem, n, widest); }

// staging capacity for the next builds (0 = unlimited)
void probe_max_stage(int v) { g_max_stage = v; }

void *probe_build(int32_t n_vars, int32_t n_polys, int64_t n_monos, const int64_t *ps,
                  const int64_t *ms, const int32_t *pos, const int32_t *exp, int L, int cc, int nt,
                  int G, char *err, int errlen)
{
    auto *t = new ScheduleTables();
    t->L = L;
    t->cc = cc;
    t->nt = nt;
    t->G = G;
    t->max_stage = g_max_stage;
    pe::CsrView v{n_vars, n_polys, n_monos, ps, ms, pos, exp};
    std::string e = pe::build_schedule_tables(v, *t);
    if (!e.empty()) {
        std::strncpy(err, e.c_str(), errlen - 1);
        err[errlen - 1] = 0;
        delete t;
        return nullptr;
    }
    return t;
}

// which: 0 word, 1 dest, 3 chunk_info,
//        6 run_info, 7 row_start, 8 group_chunk0, 12 group_info, 13 vdest
// counts only: 9 stage_slots, 10 KP, 11 MC, 14 VG, 15 max_rows
int64_t probe_count(void *h, int which)
{
    auto *t = static_cast<ScheduleTables *>(h);
    switch (which) {
    case 0: return (int64_t)t->word.size();
    case 1: return (int64_t)t->dest.size();
    case 3: return (int64_t)t->chunk_info.size();
    case 6: return (int64_t)t->run_info.size();
    case 7: return (int64_t)t->row_start.size();
    case 8: return (int64_t)t->group_chunk0.size();
    case 12: return (int64_t)t->group_info.size();
    case 13: return (int64_t)t->vdest.size();
    case 14: return t->VG;
    case 15: return t->max_rows;
    case 9: return t->stage_slots;
    case 10: return t->KP;
    case 11: return t->MC;
    }
    return -1;
}

void probe_copy(void *h, int which, void *dst)
{
    auto *t = static_cast<ScheduleTables *>(h);
    switch (which) {
    case 0: std::memcpy(dst, t->word.data(), t->word.size() * 4); break;
    case 1: std::memcpy(dst, t->dest.data(), t->dest.size() * 2); break;
    case 3: std::memcpy(dst, t->chunk_info.data(), t->chunk_info.size() * 4); break;
    case 6: std::memcpy(dst, t->run_info.data(), t->run_info.size() * 4); break;
    case 7: std::memcpy(dst, t->row_start.data(), t->row_start.size() * 2); break;
    case 8: std::memcpy(dst, t->group_chunk0.data(), t->group_chunk0.size() * 4); break;
    case 12: std::memcpy(dst, t->group_info.data(), t->group_info.size() * 4); break;
    case 13: std::memcpy(dst, t->vdest.data(), t->vdest.size() * 2); break;
    }
}

void probe_free(void *h) { delete static_cast<ScheduleTables *>(h); }
}
