// C interface of the library: system packing, schedules and launches.
//
// A system f = (C, A) (Section 2, equation (1)) arrives in CSR form and is
// validated, then packed once for the device:
//   - coefficients as [M][4] doubles (one 32-byte coalesced read per lane
//     group),
//   - per schedule (lanes per monomial L, variables per lane CC, workgroup
//     size NT, workgroups per polynomial G): a monomial-major table of
//     packed (variable, exponent-1) words padded to KP = CC*L entries, the
//     LDS staging slot of every term and the run starts of the summation.
// Tables are built on the host and uploaded once per schedule; evaluation
// calls only fill a small argument block and launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "polyeval.h"
#include "eval.hpp"
#include "internal.hpp"
#include "newton.hpp"
#include "schedule.hpp"

namespace pe {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

// a fixed buffer, so that reporting an error allocates nothing
static thread_local char g_last_error[512];

pe_status fail(pe_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
    return st;
}

pe_status hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? PE_ENOMEM : PE_EDEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------

DevBuf::~DevBuf()
{
    if (ptr) (void)hipFree(ptr);
}

hipError_t DevBuf::alloc(size_t n)
{
    if (ptr) {
        (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
    if (n == 0) return hipSuccess;
    hipError_t e = hipMalloc(&ptr, n);
    if (e == hipSuccess) bytes = n;
    return e;
}

hipError_t DevBuf::upload(const void *src, size_t n)
{
    hipError_t e = alloc(n);
    if (e != hipSuccess || n == 0) return e;
    return hipMemcpy(ptr, src, n, hipMemcpyHostToDevice);
}

// ---------------------------------------------------------------------------
// schedules
// ---------------------------------------------------------------------------

int next_pow2(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

int ilog2(int v)
{
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

size_t Schedule::lds_bytes(int words, int T, int nbuf) const
{
    const size_t np1 = (size_t)n_vars + 1;
    const size_t values = sizeof(double) * (size_t)words *
                          ((size_t)T * ((size_t)R * np1 + np1) + (size_t)nbuf * stage_slots);
    return values + sizeof(int32_t) * (size_t)nbuf * ((size_t)max_rows + 1);
}

// Build the packed tables for one schedule on the host and upload them.
static pe_status build_schedule(const System &S, Schedule &sc)
{
    ScheduleTables t;
    t.L = sc.L;
    t.cc = sc.cc;
    t.nt = sc.nt;
    t.G = sc.G;
    // staging capacity left in LDS by the power table and accumulators,
    // counted in complex double-double values (the larger precision)
    {
        const int64_t np1 = (int64_t)S.n_vars + 1;
        const int64_t R = std::max(1, S.max_exp - 1);
        // (the row table of the summation takes at most one int per
        // monomial of a chunk, plus one)
        const int64_t room = (kMaxLds - 4 * ((int64_t)sc.nt + 2)) / 32 - R * np1 - np1;
        t.max_stage = (int)std::max<int64_t>(2, std::min<int64_t>(room, 65535));
    }
    CsrView v{S.n_vars, S.n_polys, S.n_monos, S.poly_start.data(), S.mono_start.data(),
              S.pos.data(), S.exp.data()};
    std::string err = build_schedule_tables(v, t);
    if (!err.empty()) return fail(PE_EUNSUPPORTED, "%s", err.c_str());
    sc.KP = t.KP;
    sc.MC = t.MC;
    sc.VG = t.VG;
    sc.n_vars = S.n_vars;
    sc.R = std::max(1, S.max_exp - 1);
    sc.stage_slots = t.stage_slots;
    sc.max_rows = t.max_rows;
    sc.n_chunks = t.n_chunks;
    sc.any_fold = t.any_fold;
    hipError_t e;
#define PE_UP(buf)                                                                  \
    e = sc.buf.upload(t.buf.data(), t.buf.size() * sizeof(t.buf[0]));               \
    if (e != hipSuccess) return hip_fail(e, "uploading " #buf);
    PE_UP(word)
    PE_UP(dest)
    PE_UP(vdest)
    PE_UP(chunk_info)
    PE_UP(run_info)
    PE_UP(row_start)
    PE_UP(group_info)
#undef PE_UP
    return PE_OK;
}

// Automatic schedule: variables split so that each lane holds 2, 4 or 8 of
// them.  With few (polynomial, point) pairs, one workgroup takes a whole
// polynomial in a single chunk (up to 1024 lanes) so that no partial sums
// cross workgroups; otherwise workgroups of 256 lanes (512 above k = 16)
// loop over chunks.
static void auto_schedule(const System &S, int64_t n_points, int &L, int &cc, int &nt, int &G)
{
    const int k = std::max(1, S.max_k);
    if (k <= 2) {
        cc = 2;
        L = 1;
    } else if (k <= 4) {
        cc = 4;
        L = 1;
    } else if (k <= 16) {
        // eight variables per lane: measured faster than four at k = 16
        // (fewer butterfly steps, more products per lane between them)
        cc = 8;
        L = next_pow2((k + 7) / 8);
    } else {
        // four per lane above 16: a chunk of 512 lanes then stages as many
        // monomials as 256 lanes with eight, within the LDS, and sums its
        // outputs in fewer rounds (measured at k = 32, n = 512: 16% faster
        // in double-double, 14% in FP64)
        cc = 4;
        L = next_pow2((k + 3) / 4);
    }
    int64_t max_m = 0;
    for (int p = 0; p < S.n_polys; ++p)
        max_m = std::max<int64_t>(max_m, S.poly_start[p + 1] - S.poly_start[p]);
    const int64_t units = std::max<int64_t>(1, n_points) * S.n_polys;
    G = 1;
    nt = cc == 4 && k > 16 ? 512 : 256;
    if (units < 1024) {
        const int64_t lanes = std::max<int64_t>(64, max_m * L);
        nt = (int)std::min<int64_t>(1024, ((lanes + 63) / 64) * 64);
        nt = std::max(nt, 64);
    }
    // fewer lanes while a chunk's staging (at most nt / L monomials of L*cc
    // slots, plus one value slot per wave) would not fit the LDS with the
    // power table and accumulators, sized for double-double
    const int64_t np1 = (int64_t)S.n_vars + 1;
    const int64_t R = std::max(1, S.max_exp - 1);
    auto lds_need = [&](int t) {
        const int64_t slots = (int64_t)(t / L) * L * cc + t / 64 + 1;
        return 32 * (R * np1 + slots + np1);
    };
    while (nt > 64 && lds_need(nt) > kMaxLds) nt -= 64;
}

void System::schedule_key(int64_t n_points, int &L, int &cc, int &nt, int &G) const
{
    if (pin_L) {
        L = pin_L;
        cc = pin_cc;
        nt = pin_nt;
        G = pin_G;
    } else {
        auto_schedule(*this, n_points, L, cc, nt, G);
    }
}

pe_status System::schedule_for(int64_t n_points, Schedule **out)
{
    int L, cc, nt, G;
    schedule_key(n_points, L, cc, nt, G);
    return schedule_with(L, cc, nt, G, out);
}

void System::launch_shape(const Schedule &sc, int64_t n_points, bool dd, int &T, int &nbuf) const
{
    const int words = dd ? 4 : 2;
    if (pin_T || pin_nbuf) {
        T = pin_T ? pin_T : 1;
        nbuf = pin_nbuf ? pin_nbuf : 1;
        if (sc.lds_bytes(words, T, nbuf) > (size_t)kMaxLds) T = nbuf = 0;
        return;
    }
    (void)n_points;
    T = 1;
    nbuf = 1;
}

pe_status System::find_schedule(int64_t n_points, Schedule **out) const
{
    int L, cc, nt, G;
    schedule_key(n_points, L, cc, nt, G);
    for (auto &sp : schedules)
        if (sp->L == L && sp->cc == cc && sp->nt == nt && sp->G == G) {
            *out = sp.get();
            return PE_OK;
        }
    return fail(PE_EUNSUPPORTED,
                "the schedule (lanes %d, chunk_vars %d, threads %d, groups %d) for %lld points "
                "has no packed tables yet: call pe_eval_jac once with this many points first",
                L, cc, nt, G, (long long)n_points);
}

pe_status System::schedule_with(int L, int cc, int nt, int G, Schedule **out)
{
    for (auto &sp : schedules)
        if (sp->L == L && sp->cc == cc && sp->nt == nt && sp->G == G) {
            *out = sp.get();
            return PE_OK;
        }
    std::unique_ptr<Schedule> sc(new Schedule());
    sc->L = L;
    sc->cc = cc;
    sc->nt = nt;
    sc->G = G;
    pe_status st = build_schedule(*this, *sc);
    if (st != PE_OK) return st;
    *out = sc.get();
    schedules.push_back(std::move(sc));
    return PE_OK;
}

void System::fill_args(const Schedule &sc, EvalArgs &a) const
{
    a = EvalArgs{};
    a.n_vars = n_vars;
    a.n_polys = n_polys;
    a.R = sc.R;
    a.L = sc.L;
    a.log2L = ilog2(sc.L);
    a.log2VG = ilog2(sc.VG);
    // lanes per output in the summation: the largest power of two (at most
    // 16) such that every output of the chunk gets its lanes in one round
    {
        int lg = 0;
        while (lg < 4 && ((int64_t)(n_vars + 1) << (lg + 1)) <= sc.nt) ++lg;
        a.log2S = lg;
    }
    a.KP = sc.KP;
    a.G = sc.G;
    a.stage_slots = sc.stage_slots;
    a.max_rows = sc.max_rows;
    a.n_groups = n_polys * sc.G;
    a.any_fold = sc.any_fold;
    a.T = 1;
    a.nbuf = 1;
    a.word = (const uint32_t *)sc.word.ptr;
    a.dest = (const uint16_t *)sc.dest.ptr;
    a.vdest = (const uint16_t *)sc.vdest.ptr;
    a.coef = (const double *)coef.ptr;
    a.chunk_info = (const int4 *)sc.chunk_info.ptr;
    a.run_info = (const uint32_t *)sc.run_info.ptr;
    a.row_start = (const uint16_t *)sc.row_start.ptr;
    a.group_info = (const int4 *)sc.group_info.ptr;
}

pe_status System::eval_locked(int64_t n_points, const double *const x[4], double *const f[4],
                              double *const J[4], bool dd, hipStream_t hs, const int32_t *mask,
                              bool no_alloc)
{
    Schedule *sc = nullptr;
    pe_status st = no_alloc ? find_schedule(n_points, &sc) : schedule_for(n_points, &sc);
    if (st != PE_OK) return st;
    const int words = dd ? 4 : 2;
    int T = 1, nbuf = 1;
    launch_shape(*sc, n_points, dd, T, nbuf);
    if (T == 0)
        return fail(PE_EUNSUPPORTED,
                    "tiles of %d points with %d staging buffers need %zu bytes of LDS (> 160 KiB)",
                    pin_T ? pin_T : 1, pin_nbuf ? pin_nbuf : 1,
                    sc->lds_bytes(words, pin_T ? pin_T : 1, pin_nbuf ? pin_nbuf : 1));
    const size_t lds = sc->lds_bytes(words, T, nbuf);
    if (lds > kMaxLds)
        return fail(PE_EUNSUPPORTED,
                    "schedule needs %zu bytes of LDS (> 160 KiB): n_vars=%d, power rows=%d, "
                    "staging slots=%d, threads=%d",
                    lds, n_vars, sc->R, sc->stage_slots, sc->nt);

    EvalArgs a;
    fill_args(*sc, a);
    a.T = T;
    a.nbuf = nbuf;
    a.n_points = n_points;
    for (int q = 0; q < 4; ++q) {
        a.x[q] = x[q];
        a.f[q] = f[q];
        a.J[q] = J[q];
    }
    a.mask = mask;

    if (sc->G > 1) {
        if ((int64_t)(n_vars + 1) * n_polys >= ((int64_t)1 << 31))
            return fail(PE_EUNSUPPORTED, "groups > 1 needs (n_vars+1)*n_polys < 2^31");
        const size_t need_part =
            (size_t)n_points * a.n_groups * ((size_t)n_vars + 1) * words * sizeof(double);
        if (no_alloc) {
            if (need_part > kStaticScratchBytes)
                return fail(PE_EUNSUPPORTED,
                            "%lld points need %zu bytes of partial rows (groups = %d), more "
                            "than the %zu bytes of the static scratch",
                            (long long)n_points, need_part, sc->G, kStaticScratchBytes);
            a.partial = (double *)static_scratch_ptr(device);
            if (!a.partial) return fail(PE_EDEVICE, "no static scratch on device %d", device);
        } else if (partial.bytes < need_part) {
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            if (hipStreamIsCapturing(hs, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
                return fail(PE_EUNSUPPORTED,
                            "scratch must grow during stream capture: call once before capturing");
            (void)hipStreamSynchronize(hs);
            hipError_t e = partial.alloc(need_part);
            if (e != hipSuccess) return hip_fail(e, "allocating partial sums");
        }
        if (!no_alloc) a.partial = (double *)partial.ptr;
    }
    const int maxt = sc->nt <= 256 ? 256 : (sc->nt <= 512 ? 512 : 1024);
    const int64_t gy = std::min<int64_t>((n_points + T - 1) / T, 65535);
    dim3 grid((unsigned)a.n_groups, (unsigned)gy, 1);
    dim3 block((unsigned)sc->nt, 1, 1);
    hipError_t e = launch_eval(dd ? 1 : 0, sc->cc, maxt, a, grid, block, lds, hs);
    if (e != hipSuccess) return hip_fail(e, "launching the evaluation kernel");
    if (sc->G > 1) {
        e = launch_combine(dd ? 1 : 0, a, hs);
        if (e != hipSuccess) return hip_fail(e, "launching the combination kernel");
    }
    return PE_OK;
}

static std::once_flag g_init_once;
static hipError_t g_init_err = hipSuccess;

hipError_t library_init()
{
    std::call_once(g_init_once, [] {
        g_init_err = eval_kernels_init();
        if (g_init_err == hipSuccess) g_init_err = newton_kernels_init();
    });
    return g_init_err;
}

}  // namespace pe

using namespace pe;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

const char *pe_version(void) { return "polyeval 0.1 (gfx950)"; }

const char *pe_last_error(void) { return g_last_error; }

pe_status pe_create_system(int32_t n_vars, int32_t n_polys, int64_t n_monos,
                           const int64_t *poly_start, const int64_t *mono_start,
                           const int32_t *pos, const int32_t *exp, pe_cvec coef, pe_system *out)
{
    if (!out) return fail(PE_EINVAL, "pe_create_system: out is NULL");
    *out = nullptr;
    if (n_vars < 1 || n_vars >= (1 << 24)) return fail(PE_EINVAL, "n_vars = %d out of range", n_vars);
    if (n_polys < 1) return fail(PE_EINVAL, "n_polys = %d must be >= 1", n_polys);
    if (n_monos < 0) return fail(PE_EINVAL, "n_monos = %lld must be >= 0", (long long)n_monos);
    if (!poly_start || !mono_start) return fail(PE_EINVAL, "poly_start / mono_start is NULL");
    if (n_monos > 0 && (!coef.re_hi || !coef.re_lo || !coef.im_hi || !coef.im_lo))
        return fail(PE_EINVAL, "a coefficient plane is NULL");
    if (poly_start[0] != 0) return fail(PE_EINVAL, "poly_start[0] must be 0");
    for (int32_t p = 0; p < n_polys; ++p)
        if (poly_start[p + 1] < poly_start[p])
            return fail(PE_EINVAL, "poly_start decreases at polynomial %d", p);
    if (poly_start[n_polys] != n_monos)
        return fail(PE_EINVAL, "poly_start[n_polys] = %lld != n_monos = %lld",
                    (long long)poly_start[n_polys], (long long)n_monos);
    if (mono_start[0] != 0) return fail(PE_EINVAL, "mono_start[0] must be 0");
    for (int64_t s = 0; s < n_monos; ++s)
        if (mono_start[s + 1] < mono_start[s])
            return fail(PE_EINVAL, "mono_start decreases at monomial %lld", (long long)s);
    const int64_t nnz = mono_start[n_monos];
    if (nnz > 0 && (!pos || !exp)) return fail(PE_EINVAL, "pos / exp is NULL");
    int max_k = 0, max_exp = 1;
    for (int64_t s = 0; s < n_monos; ++s) {
        const int64_t b = mono_start[s], e = mono_start[s + 1];
        if (e - b > 256) return fail(PE_EUNSUPPORTED, "monomial %lld has %lld > 256 variables",
                                     (long long)s, (long long)(e - b));
        max_k = std::max(max_k, (int)(e - b));
        for (int64_t j = b; j < e; ++j) {
            if (pos[j] < 0 || pos[j] >= n_vars)
                return fail(PE_EINVAL, "monomial %lld: variable index %d out of range [0, %d)",
                            (long long)s, pos[j], n_vars);
            if (j > b && pos[j] <= pos[j - 1])
                return fail(PE_EINVAL, "monomial %lld: variable indices not strictly increasing",
                            (long long)s);
            if (exp[j] < 1 || exp[j] > 256)
                return fail(PE_EINVAL, "monomial %lld: exponent %d out of range [1, 256]",
                            (long long)s, exp[j]);
            max_exp = std::max(max_exp, (int)exp[j]);
        }
        const double c4[4] = {coef.re_hi[s], coef.re_lo[s], coef.im_hi[s], coef.im_lo[s]};
        for (double v : c4)
            if (!std::isfinite(v))
                return fail(PE_EINVAL, "monomial %lld: coefficient is not finite", (long long)s);
    }
    hipError_t he = library_init();
    if (he != hipSuccess) return hip_fail(he, "initializing kernels");

    std::unique_ptr<System> S(new System());
    S->n_vars = n_vars;
    S->n_polys = n_polys;
    S->n_monos = n_monos;
    S->max_k = max_k;
    S->max_exp = max_exp;
    S->poly_start.assign(poly_start, poly_start + n_polys + 1);
    S->mono_start.assign(mono_start, mono_start + n_monos + 1);
    if (nnz) {
        S->pos.assign(pos, pos + nnz);
        S->exp.assign(exp, exp + nnz);
    }
    std::vector<double> c((size_t)n_monos * 4);
    for (int64_t s = 0; s < n_monos; ++s) {
        c[4 * s + 0] = coef.re_hi[s];
        c[4 * s + 1] = coef.re_lo[s];
        c[4 * s + 2] = coef.im_hi[s];
        c[4 * s + 3] = coef.im_lo[s];
    }
    if (hipGetDevice(&S->device) != hipSuccess) return fail(PE_EDEVICE, "hipGetDevice failed");
    // the device address of the static scratch, looked up once per device
    he = static_scratch_setup();
    if (he != hipSuccess) return hip_fail(he, "locating the static scratch");
    he = S->coef.upload(c.data(), c.size() * sizeof(double));
    if (he != hipSuccess) return hip_fail(he, "uploading coefficients");
    if (nnz >= ((int64_t)1 << 31)) return fail(PE_EUNSUPPORTED, "more than 2^31 support entries");
    {
        std::vector<int32_t> ms32((size_t)n_monos + 1);
        for (int64_t s = 0; s <= n_monos; ++s) ms32[(size_t)s] = (int32_t)mono_start[s];
        std::vector<uint32_t> w((size_t)nnz);
        for (int64_t j = 0; j < nnz; ++j) w[(size_t)j] = pack_word(pos[j], exp[j]);
        he = S->d_poly_start.upload(poly_start, sizeof(int64_t) * ((size_t)n_polys + 1));
        if (he == hipSuccess) he = S->d_mono_start.upload(ms32.data(), ms32.size() * sizeof(int32_t));
        if (he == hipSuccess && nnz) he = S->d_word.upload(w.data(), w.size() * sizeof(uint32_t));
        if (he != hipSuccess) return hip_fail(he, "uploading residual tables");
    }
    *out = reinterpret_cast<pe_system>(S.release());
    return PE_OK;
}

pe_status pe_destroy_system(pe_system sys)
{
    delete reinterpret_cast<System *>(sys);
    return PE_OK;
}

pe_status pe_system_info(pe_system sys, int32_t *n_vars, int32_t *n_polys, int64_t *n_monos,
                         int32_t *max_k, int32_t *max_exp)
{
    if (!sys) return fail(PE_EINVAL, "NULL system");
    const System *S = reinterpret_cast<System *>(sys);
    if (n_vars) *n_vars = S->n_vars;
    if (n_polys) *n_polys = S->n_polys;
    if (n_monos) *n_monos = S->n_monos;
    if (max_k) *max_k = S->max_k;
    if (max_exp) *max_exp = S->max_exp;
    return PE_OK;
}

pe_status pe_set_schedule(pe_system sys, int32_t lanes, int32_t chunk_vars, int32_t threads,
                          int32_t groups, int32_t tile_points, int32_t stage_buffers)
{
    if (!sys) return fail(PE_EINVAL, "NULL system");
    System *S = reinterpret_cast<System *>(sys);
    if (tile_points < 0 || tile_points > 32)
        return fail(PE_EINVAL, "tile_points = %d must be in [0, 32]", tile_points);
    if (stage_buffers < 0 || stage_buffers > 2)
        return fail(PE_EINVAL, "stage_buffers = %d must be 0, 1 or 2", stage_buffers);
    std::lock_guard<std::mutex> lock(S->mu);
    if (lanes == 0 && chunk_vars == 0 && threads == 0 && groups == 0) {
        S->pin_L = S->pin_cc = S->pin_nt = S->pin_G = 0;
        S->pin_T = tile_points;
        S->pin_nbuf = stage_buffers;
        return PE_OK;
    }
    if (lanes < 1 || lanes > 32 || (lanes & (lanes - 1)))
        return fail(PE_EINVAL, "lanes = %d must be a power of two in [1, 32]", lanes);
    if (chunk_vars != 2 && chunk_vars != 4 && chunk_vars != 8)
        return fail(PE_EINVAL, "chunk_vars = %d must be 2, 4 or 8", chunk_vars);
    if (threads < 64 || threads > 1024 || threads % 64)
        return fail(PE_EINVAL, "threads = %d must be a multiple of 64 in [64, 1024]", threads);
    if (groups < 1) return fail(PE_EINVAL, "groups = %d must be >= 1", groups);
    if (lanes * chunk_vars < S->max_k)
        return fail(PE_EINVAL, "lanes*chunk_vars = %d below the largest monomial size %d",
                    lanes * chunk_vars, S->max_k);
    S->pin_L = lanes;
    S->pin_cc = chunk_vars;
    S->pin_nt = threads;
    S->pin_G = groups;
    S->pin_T = tile_points;
    S->pin_nbuf = stage_buffers;
    return PE_OK;
}

pe_status pe_get_schedule(pe_system sys, int64_t n_points, int32_t *lanes, int32_t *chunk_vars,
                          int32_t *threads, int32_t *groups, int32_t *tile_points,
                          int32_t *stage_buffers)
{
    if (!sys) return fail(PE_EINVAL, "NULL system");
    System *S = reinterpret_cast<System *>(sys);
    std::lock_guard<std::mutex> lock(S->mu);
    int L, cc, nt, G;
    S->schedule_key(n_points, L, cc, nt, G);
    if (lanes) *lanes = L;
    if (chunk_vars) *chunk_vars = cc;
    if (threads) *threads = nt;
    if (groups) *groups = G;
    if (tile_points || stage_buffers) {
        // the tile shape depends on the schedule's tables (their LDS size)
        Schedule *sc = nullptr;
        pe_status st = S->schedule_for(n_points, &sc);
        if (st != PE_OK) return st;
        int T = 1, nbuf = 1;
        S->launch_shape(*sc, n_points, true, T, nbuf);
        if (tile_points) *tile_points = T;
        if (stage_buffers) *stage_buffers = nbuf;
    }
    return PE_OK;
}

static pe_status eval_jac_entry(pe_system sys, int64_t n_points, pe_cvec points, pe_cvec out_f,
                                pe_cvec out_J, pe_precision precision, void *stream, bool no_alloc)
{
    if (!sys) return fail(PE_EINVAL, "NULL system");
    if (n_points < 0) return fail(PE_EINVAL, "n_points = %lld < 0", (long long)n_points);
    if (precision != PE_FP64 && precision != PE_DD) return fail(PE_EINVAL, "unknown precision");
    System *S = reinterpret_cast<System *>(sys);
    if (n_points == 0) return PE_OK;
    const bool dd = precision == PE_DD;
    if (!points.re_hi || !points.im_hi || (dd && (!points.re_lo || !points.im_lo)))
        return fail(PE_EINVAL, "a required point plane is NULL");
    if (!out_f.re_hi || !out_f.im_hi || (dd && (!out_f.re_lo || !out_f.im_lo)))
        return fail(PE_EINVAL, "a required value plane is NULL");
    const bool jac = out_J.re_hi || out_J.re_lo || out_J.im_hi || out_J.im_lo;
    if (jac && (!out_J.re_hi || !out_J.im_hi || (dd && (!out_J.re_lo || !out_J.im_lo))))
        return fail(PE_EINVAL, "out_J is partially NULL");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != S->device)
        return fail(PE_EINVAL, "the current device (%d) is not the system's device (%d)", dev,
                    S->device);
    const double *x[4] = {points.re_hi, points.re_lo, points.im_hi, points.im_lo};
    double *f[4] = {out_f.re_hi, out_f.re_lo, out_f.im_hi, out_f.im_lo};
    double *J[4] = {jac ? out_J.re_hi : nullptr, out_J.re_lo, out_J.im_hi, out_J.im_lo};
    std::lock_guard<std::mutex> lock(S->mu);
    return S->eval_locked(n_points, x, f, J, dd, reinterpret_cast<hipStream_t>(stream), nullptr,
                          no_alloc);
}

pe_status pe_eval_jac(pe_system sys, int64_t n_points, pe_cvec points, pe_cvec out_f,
                      pe_cvec out_J, pe_precision precision, void *stream)
{
    return eval_jac_entry(sys, n_points, points, out_f, out_J, precision, stream, false);
}

pe_status pe_eval_jac_noalloc(pe_system sys, int64_t n_points, pe_cvec points, pe_cvec out_f,
                              pe_cvec out_J, pe_precision precision, void *stream)
{
    return eval_jac_entry(sys, n_points, points, out_f, out_J, precision, stream, true);
}

pe_status pe_eval_jac_qd(pe_system sys, int64_t n_points, const double *const *points,
                         double *const *out_f, double *const *out_J, void *stream)
{
    if (!sys) return fail(PE_EINVAL, "NULL system");
    if (n_points < 0) return fail(PE_EINVAL, "n_points = %lld < 0", (long long)n_points);
    System *S = reinterpret_cast<System *>(sys);
    if (n_points == 0) return PE_OK;
    if (!points || !out_f) return fail(PE_EINVAL, "NULL plane array");
    bool jac = out_J != nullptr;
    for (int q = 0; q < 8; ++q) {
        if (!points[q]) return fail(PE_EINVAL, "point plane %d is NULL", q);
        if (!out_f[q]) return fail(PE_EINVAL, "value plane %d is NULL", q);
        if (jac && !out_J[q]) return fail(PE_EINVAL, "Jacobian plane %d is NULL", q);
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != S->device)
        return fail(PE_EINVAL, "the current device (%d) is not the system's device (%d)", dev,
                    S->device);
    std::lock_guard<std::mutex> lock(S->mu);
    // quad-double values take eight registers: four variables per lane fill
    // a SIMD with one wave of 256 threads, two per lane leave room for two
    // waves (512 threads) at the same monomials per chunk.  With fewer
    // (polynomial, point) pairs than compute units, each polynomial is split
    // over G = 2 or 4 workgroups whose partial rows are added by the
    // combination kernel.
    const int k = std::max(1, S->max_k);
    int cc = k <= 2 ? 2 : 4;
    int L = next_pow2((k + cc - 1) / cc);
    if (L > 32) return fail(PE_EUNSUPPORTED, "monomials of more than 128 variables in quad-double");
    // two variables per lane on 512 threads keep the same monomials per chunk
    // with two waves per SIMD, when lanes (L <= 32) and LDS allow
    int nt = 256;
    if (cc == 4 && 2 * L <= 32) {
        cc = 2;
        L *= 2;
        nt = 512;
    }
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    int64_t max_m = 0;
    for (int p = 0; p < S->n_polys; ++p)
        max_m = std::max<int64_t>(max_m, S->poly_start[(size_t)p + 1] - S->poly_start[(size_t)p]);
    const int64_t mc = nt / L;  // monomials per chunk
    const int64_t max_chunks = (max_m + mc - 1) / mc;
    const int64_t pairs = (int64_t)S->n_polys * n_points;
    int G = 1;
    while (G < 4 && 2 * G <= max_chunks && pairs * G < cus) G *= 2;
    if ((int64_t)(S->n_vars + 1) * S->n_polys >= ((int64_t)1 << 31)) G = 1;
    Schedule *sc = nullptr;
    pe_status st = S->schedule_with(L, cc, nt, G, &sc);
    if (st != PE_OK) return st;
    if (nt == 512 && sc->lds_bytes(8) > kMaxLds) {
        cc = 4;
        L /= 2;
        nt = 256;
        st = S->schedule_with(L, cc, nt, G, &sc);
        if (st != PE_OK) return st;
    }
    const size_t lds = sc->lds_bytes(8);
    if (lds > kMaxLds)
        return fail(PE_EUNSUPPORTED,
                    "quad-double needs %zu bytes of LDS (> 160 KiB): n_vars=%d, power rows=%d, "
                    "staging slots=%d",
                    lds, S->n_vars, sc->R, sc->stage_slots);
    EvalArgs a;
    S->fill_args(*sc, a);
    a.n_points = n_points;
    for (int q = 0; q < 8; ++q) {
        a.x[q] = points[q];
        a.f[q] = out_f[q];
        a.J[q] = jac ? out_J[q] : nullptr;
    }
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    if (sc->G > 1) {
        // eight doubles per complex quad-double entry
        const size_t need_part =
            (size_t)n_points * a.n_groups * ((size_t)S->n_vars + 1) * 8 * sizeof(double);
        if (S->partial.bytes < need_part) {
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            if (hipStreamIsCapturing(hs, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
                return fail(PE_EUNSUPPORTED,
                            "scratch must grow during stream capture: call once before capturing");
            (void)hipStreamSynchronize(hs);
            hipError_t e = S->partial.alloc(need_part);
            if (e != hipSuccess) return hip_fail(e, "allocating partial sums");
        }
        a.partial = (double *)S->partial.ptr;
    }
    const int64_t gy = std::min<int64_t>(n_points, 65535);
    dim3 grid((unsigned)a.n_groups, (unsigned)gy, 1);
    hipError_t e = launch_eval(2, cc, nt, a, grid, dim3((unsigned)nt), lds, hs);
    if (e != hipSuccess) return hip_fail(e, "launching the quad-double evaluation");
    if (sc->G > 1) {
        e = launch_combine(2, a, hs);
        if (e != hipSuccess) return hip_fail(e, "launching the combination kernel");
    }
    return PE_OK;
}

}  // extern "C"
