// Batched evaluation of many systems in one persistent launch, and the
// autotuner that picks its schedule (C interface).
//
// The paper evaluates one system at one point per launch sequence
// (Section 4: three kernels per evaluation).  Here a batch packs several
// systems of different n, m and k; one launch of the persistent batch kernel
// walks a task list (system, point, range of polynomials) ordered longest
// first, each workgroup taking every gridDim-th task.  The launch contains no
// allocation, copy or memset, so it can be captured in a hipGraph and
// replayed.  The schedule -- variables per lane, workgroup size, lanes per
// monomial, task size -- is chosen by timing candidates on the caller's
// buffers (pe_autotune_batch), optionally cached in a text file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "polyeval.h"
#include "eval.hpp"
#include "internal.hpp"

using namespace pe;

namespace pe {

struct BatchConfig {
    int cc = 4;          // variables per lane (template)
    int nt = 256;        // lanes per workgroup
    int lanes_mult = 1;  // lanes per monomial = minimal power of two for k, times this
    int task_terms = 16384;  // target derivative terms per task
    bool operator==(const BatchConfig &o) const
    {
        return cc == o.cc && nt == o.nt && lanes_mult == o.lanes_mult && task_terms == o.task_terms;
    }
};

struct Batch {
    std::vector<System *> sys;
    int device = 0;
    BatchConfig cfg;
    bool tuned = false;
    // built state
    bool built = false;
    BatchConfig built_cfg;
    std::vector<int64_t> built_pps;
    int64_t n_tasks = 0;
    size_t lds_dd = 0, lds_64 = 0;
    int grid = 0;
    DevBuf desc, tasks;
    std::mutex mu;
};

static int lanes_for(int k, const BatchConfig &c)
{
    int L = next_pow2(std::max(1, (std::max(1, k) + c.cc - 1) / c.cc)) * c.lanes_mult;
    return std::min(L, 32);
}

// (Re)build descriptors and tasks for `pps` points per system.
static pe_status build_batch(Batch &B, const std::vector<int64_t> &pps, hipStream_t hs)
{
    const int ns = (int)B.sys.size();
    std::vector<BatchDesc> descs((size_t)ns);
    struct HostTask {
        BatchTask t;
        double cost;
    };
    std::vector<HostTask> tasks;
    int64_t x_off = 0, f_off = 0, J_off = 0;
    size_t lds_max = 0;
    for (int i = 0; i < ns; ++i) {
        System &S = *B.sys[i];
        const int L = lanes_for(S.max_k, B.cfg);
        Schedule *sc = nullptr;
        pe_status st = S.schedule_with(L, B.cfg.cc, B.cfg.nt, 1, &sc);
        if (st != PE_OK) return st;
        S.fill_args(*sc, descs[(size_t)i].a);
        descs[(size_t)i].a.n_points = pps[(size_t)i];
        descs[(size_t)i].x_off = x_off;
        descs[(size_t)i].f_off = f_off;
        descs[(size_t)i].J_off = J_off;
        x_off += pps[(size_t)i] * S.n_vars;
        f_off += pps[(size_t)i] * S.n_polys;
        J_off += pps[(size_t)i] * (int64_t)S.n_vars * S.n_polys;
        lds_max = std::max(lds_max, sc->lds_bytes(4));
        // polynomial ranges of about task_terms derivative terms
        std::vector<int> cut{0};
        int64_t acc = 0;
        for (int p = 0; p < S.n_polys; ++p) {
            acc += S.mono_start[S.poly_start[p + 1]] - S.mono_start[S.poly_start[p]] +
                   (S.poly_start[p + 1] - S.poly_start[p]);
            if (acc >= B.cfg.task_terms) {
                cut.push_back(p + 1);
                acc = 0;
            }
        }
        if (cut.back() != S.n_polys) cut.push_back(S.n_polys);
        for (int64_t pt = 0; pt < pps[(size_t)i]; ++pt)
            for (size_t r = 0; r + 1 < cut.size(); ++r) {
                const int p0 = cut[r], p1 = cut[r + 1];
                double cost = (double)S.n_vars * sc->R;  // power table
                for (int p = p0; p < p1; ++p) {
                    const int64_t mp = S.poly_start[p + 1] - S.poly_start[p];
                    cost += (double)mp * (6.0 * std::max(1, S.max_k) - 5.0) + S.n_vars;
                }
                tasks.push_back({{i, p0, p1, 0, pt}, cost});
            }
    }
    if (lds_max > kMaxLds)
        return fail(PE_EUNSUPPORTED, "a system of the batch needs %zu bytes of LDS", lds_max);
    std::stable_sort(tasks.begin(), tasks.end(),
                     [](const HostTask &a, const HostTask &b) { return a.cost > b.cost; });
    std::vector<BatchTask> tv(tasks.size());
    for (size_t j = 0; j < tasks.size(); ++j) tv[j] = tasks[j].t;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(hs, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return fail(PE_EUNSUPPORTED,
                    "the batch tables must be built before capture: call once outside capture");
    (void)hipStreamSynchronize(hs);
    hipError_t e = B.desc.upload(descs.data(), descs.size() * sizeof(BatchDesc));
    if (e == hipSuccess) e = B.tasks.upload(tv.data(), tv.size() * sizeof(BatchTask));
    if (e != hipSuccess) return hip_fail(e, "uploading batch tables");
    B.n_tasks = (int64_t)tv.size();
    B.lds_dd = lds_max;
    B.lds_64 = lds_max / 2;
    // persistent grid: as many workgroups as fit on the chip at once
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    }
    const int maxt = B.cfg.nt <= 256 ? 256 : (B.cfg.nt <= 512 ? 512 : 1024);
    const int per_cu = batch_occupancy(1, B.cfg.cc, maxt, B.cfg.nt, lds_max);
    B.grid = (int)std::min<int64_t>(B.n_tasks, (int64_t)cus * per_cu);
    B.built = true;
    B.built_cfg = B.cfg;
    B.built_pps = pps;
    return PE_OK;
}

static pe_status launch_batch_eval(Batch &B, const std::vector<int64_t> &pps, pe_cvec points,
                                   pe_cvec out_f, pe_cvec out_J, bool dd, hipStream_t hs)
{
    if (!B.built || !(B.built_cfg == B.cfg) || B.built_pps != pps) {
        pe_status st = build_batch(B, pps, hs);
        if (st != PE_OK) return st;
    }
    if (B.n_tasks == 0) return PE_OK;
    BatchArgs a{};
    a.desc = (const BatchDesc *)B.desc.ptr;
    a.tasks = (const BatchTask *)B.tasks.ptr;
    a.n_tasks = B.n_tasks;
    const bool jac = out_J.re_hi != nullptr;
    const double *x[4] = {points.re_hi, points.re_lo, points.im_hi, points.im_lo};
    double *f[4] = {out_f.re_hi, out_f.re_lo, out_f.im_hi, out_f.im_lo};
    double *J[4] = {out_J.re_hi, out_J.re_lo, out_J.im_hi, out_J.im_lo};
    for (int q = 0; q < 4; ++q) {
        a.x[q] = x[q];
        a.f[q] = f[q];
        a.J[q] = jac ? J[q] : nullptr;
    }
    const int maxt = B.cfg.nt <= 256 ? 256 : (B.cfg.nt <= 512 ? 512 : 1024);
    hipError_t e = launch_batch(dd ? 1 : 0, B.cfg.cc, maxt, a, dim3((unsigned)B.grid),
                                dim3((unsigned)B.cfg.nt), dd ? B.lds_dd : B.lds_64, hs);
    if (e != hipSuccess) return hip_fail(e, "launching the batch kernel");
    return PE_OK;
}

static std::string batch_key(const Batch &B, const std::vector<int64_t> &pps, bool dd)
{
    std::ostringstream k;
    k << "batch" << (dd ? "-dd" : "-f64");
    for (size_t i = 0; i < B.sys.size(); ++i) {
        const System &S = *B.sys[i];
        k << ":" << S.n_vars << "x" << S.n_polys << "x" << S.n_monos << "k" << S.max_k << "d"
          << S.max_exp << "p" << pps[i];
    }
    return k.str();
}

static bool cache_lookup(const char *path, const std::string &key, std::vector<int> &vals)
{
    if (!path || !*path) return false;
    std::ifstream in(path);
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {
        const size_t sp = line.find(' ');
        if (sp == std::string::npos || line.compare(0, sp, key) != 0 || sp != key.size()) continue;
        std::istringstream is(line.substr(sp + 1));
        std::vector<int> v;
        int x;
        while (is >> x) v.push_back(x);
        vals = v;
        found = true;  // the last entry for a key wins
    }
    return found;
}

static void cache_store(const char *path, const std::string &key, const std::vector<int> &vals)
{
    if (!path || !*path) return;
    std::ofstream out(path, std::ios::app);
    out << key;
    for (int v : vals) out << ' ' << v;
    out << '\n';
}

static std::vector<int64_t> pps_vec(const Batch &B, const int64_t *points_per_system)
{
    return std::vector<int64_t>(points_per_system, points_per_system + B.sys.size());
}

// Milliseconds per call of fn(stream).  One untimed eager call on hs (it
// builds tables and grows scratch), then `reps` calls captured in a hipGraph
// on a private stream whose replays are timed with events, best of three, so
// the host's launch rate does not enter the figure (as for callers that
// replay graphs).  If the calls cannot be captured, eager calls on hs are
// timed instead.
template <class F>
static pe_status time_calls(hipStream_t hs, int reps, F fn, float &ms)
{
    pe_status st = fn(hs);
    if (st != PE_OK) return st;
    if (hipStreamSynchronize(hs) != hipSuccess) return fail(PE_EDEVICE, "stream synchronize failed");
    reps = std::max(1, reps);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(PE_EDEVICE, "hipEventCreate failed");
    }
    float best = -1.f;
    hipStream_t ts = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (hipStreamCreateWithFlags(&ts, hipStreamNonBlocking) == hipSuccess &&
        hipStreamBeginCapture(ts, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        pe_status cst = PE_OK;
        for (int r = 0; r < reps && cst == PE_OK; ++r) cst = fn(ts);
        const hipError_t ce = hipStreamEndCapture(ts, &graph);
        if (cst == PE_OK && ce == hipSuccess && graph &&
            hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess &&
            hipGraphLaunch(exec, ts) == hipSuccess && hipStreamSynchronize(ts) == hipSuccess) {
            for (int k = 0; k < 3; ++k) {
                float t = 0.f;
                if (hipEventRecord(e0, ts) != hipSuccess || hipGraphLaunch(exec, ts) != hipSuccess ||
                    hipEventRecord(e1, ts) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
                    best = -1.f;
                    break;
                }
                if (best < 0.f || t < best) best = t;
            }
        }
        (void)hipGetLastError();  // a failed capture leaves its error behind
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (ts) {
        (void)hipStreamSynchronize(ts);
        (void)hipStreamDestroy(ts);
    }
    if (best < 0.f) {
        (void)hipEventRecord(e0, hs);
        for (int r = 0; r < reps && st == PE_OK; ++r) st = fn(hs);
        (void)hipEventRecord(e1, hs);
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(&best, e0, e1);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ms = best / reps;
    return st;
}

}  // namespace pe

extern "C" {

pe_status pe_create_batch(const pe_system *systems, int32_t count, pe_batch *out)
{
    if (!out) return fail(PE_EINVAL, "out is NULL");
    *out = nullptr;
    if (!systems || count < 1) return fail(PE_EINVAL, "need at least one system");
    std::unique_ptr<Batch> B(new Batch());
    for (int32_t i = 0; i < count; ++i) {
        if (!systems[i]) return fail(PE_EINVAL, "system %d is NULL", i);
        System *S = reinterpret_cast<System *>(systems[i]);
        if (i > 0 && S->device != B->device)
            return fail(PE_EINVAL, "systems of a batch must live on one device");
        B->device = S->device;
        B->sys.push_back(S);
    }
    *out = reinterpret_cast<pe_batch>(B.release());
    return PE_OK;
}

pe_status pe_destroy_batch(pe_batch b)
{
    delete reinterpret_cast<Batch *>(b);
    return PE_OK;
}

pe_status pe_batch_layout(pe_batch b, const int64_t *points_per_system, int64_t *points_offset,
                          int64_t *f_offset, int64_t *J_offset)
{
    if (!b || !points_per_system) return fail(PE_EINVAL, "NULL argument");
    Batch *B = reinterpret_cast<Batch *>(b);
    int64_t xo = 0, fo = 0, Jo = 0;
    for (size_t i = 0; i <= B->sys.size(); ++i) {
        if (points_offset) points_offset[i] = xo;
        if (f_offset) f_offset[i] = fo;
        if (J_offset) J_offset[i] = Jo;
        if (i == B->sys.size()) break;
        const System &S = *B->sys[i];
        if (points_per_system[i] < 0) return fail(PE_EINVAL, "negative point count");
        xo += points_per_system[i] * S.n_vars;
        fo += points_per_system[i] * S.n_polys;
        Jo += points_per_system[i] * (int64_t)S.n_vars * S.n_polys;
    }
    return PE_OK;
}

pe_status pe_eval_jac_batch(pe_batch b, const int64_t *points_per_system, pe_cvec points,
                            pe_cvec out_f, pe_cvec out_J, pe_precision precision, void *stream)
{
    if (!b || !points_per_system) return fail(PE_EINVAL, "NULL argument");
    if (precision != PE_FP64 && precision != PE_DD) return fail(PE_EINVAL, "unknown precision");
    Batch *B = reinterpret_cast<Batch *>(b);
    const bool dd = precision == PE_DD;
    if (!points.re_hi || !points.im_hi || (dd && (!points.re_lo || !points.im_lo)))
        return fail(PE_EINVAL, "a required point plane is NULL");
    if (!out_f.re_hi || !out_f.im_hi || (dd && (!out_f.re_lo || !out_f.im_lo)))
        return fail(PE_EINVAL, "a required value plane is NULL");
    const bool jac = out_J.re_hi || out_J.re_lo || out_J.im_hi || out_J.im_lo;
    if (jac && (!out_J.re_hi || !out_J.im_hi || (dd && (!out_J.re_lo || !out_J.im_lo))))
        return fail(PE_EINVAL, "out_J is partially NULL");
    for (size_t i = 0; i < B->sys.size(); ++i)
        if (points_per_system[i] < 0) return fail(PE_EINVAL, "negative point count");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != B->device)
        return fail(PE_EINVAL, "the current device is not the batch's device");
    std::lock_guard<std::mutex> lock(B->mu);
    return launch_batch_eval(*B, pps_vec(*B, points_per_system), points, out_f, out_J, dd,
                             reinterpret_cast<hipStream_t>(stream));
}

pe_status pe_batch_config(pe_batch b, int32_t *chunk_vars, int32_t *threads, int32_t *lanes_mult,
                          int32_t *task_terms)
{
    if (!b) return fail(PE_EINVAL, "NULL batch");
    Batch *B = reinterpret_cast<Batch *>(b);
    if (chunk_vars) *chunk_vars = B->cfg.cc;
    if (threads) *threads = B->cfg.nt;
    if (lanes_mult) *lanes_mult = B->cfg.lanes_mult;
    if (task_terms) *task_terms = B->cfg.task_terms;
    return PE_OK;
}

pe_status pe_autotune_batch(pe_batch b, const int64_t *points_per_system, pe_cvec points,
                            pe_cvec out_f, pe_cvec out_J, pe_precision precision, void *stream,
                            const char *cache_path)
{
    if (!b || !points_per_system) return fail(PE_EINVAL, "NULL argument");
    Batch *B = reinterpret_cast<Batch *>(b);
    const bool dd = precision == PE_DD;
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    const std::vector<int64_t> pps = pps_vec(*B, points_per_system);
    const std::string key = batch_key(*B, pps, dd);
    std::vector<int> cached;
    {
        std::lock_guard<std::mutex> lock(B->mu);
        if (cache_lookup(cache_path, key, cached) && cached.size() == 4) {
            B->cfg = {cached[0], cached[1], cached[2], cached[3]};
            B->tuned = true;
            return PE_OK;
        }
    }
    std::vector<BatchConfig> cands;
    for (int cc : {2, 4, 8})
        for (int nt : {256, 512})
            for (int lm : {1, 2})
                for (int tt : {4096, 32768}) cands.push_back({cc, nt, lm, tt});
    float best = -1.f;
    BatchConfig best_cfg = B->cfg;
    for (const BatchConfig &c : cands) {
        std::lock_guard<std::mutex> lock(B->mu);
        B->cfg = c;
        float ms = 0.f;
        pe_status st = time_calls(hs, 2, [&](hipStream_t ts) {
            return launch_batch_eval(*B, pps, points, out_f, out_J, dd, ts);
        }, ms);
        if (st == PE_EUNSUPPORTED) continue;  // e.g. LDS too large for this schedule
        if (st != PE_OK) return st;
        if (best < 0.f || ms < best) {
            best = ms;
            best_cfg = c;
        }
    }
    if (best < 0.f) return fail(PE_EUNSUPPORTED, "no batch schedule fits");
    std::lock_guard<std::mutex> lock(B->mu);
    B->cfg = best_cfg;
    B->tuned = true;
    cache_store(cache_path, key, {best_cfg.cc, best_cfg.nt, best_cfg.lanes_mult, best_cfg.task_terms});
    return PE_OK;
}

pe_status pe_autotune_system(pe_system sys, int64_t n_points, pe_cvec points, pe_cvec out_f,
                             pe_cvec out_J, pe_precision precision, void *stream,
                             const char *cache_path)
{
    if (!sys) return fail(PE_EINVAL, "NULL system");
    if (n_points < 1) return fail(PE_EINVAL, "n_points must be >= 1");
    System *S = reinterpret_cast<System *>(sys);
    const bool dd = precision == PE_DD;
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    std::ostringstream ks;
    ks << "system" << (dd ? "-dd" : "-f64") << ":" << S->n_vars << "x" << S->n_polys << "x"
       << S->n_monos << "k" << S->max_k << "d" << S->max_exp << "p" << n_points;
    const std::string key = ks.str();
    std::vector<int> cached;
    if (cache_lookup(cache_path, key, cached) && cached.size() == 6)
        return pe_set_schedule(sys, cached[0], cached[1], cached[2], cached[3], cached[4],
                               cached[5]);
    const double *x[4] = {points.re_hi, points.re_lo, points.im_hi, points.im_lo};
    double *f[4] = {out_f.re_hi, out_f.re_lo, out_f.im_hi, out_f.im_lo};
    double *J[4] = {out_J.re_hi, out_J.re_lo, out_J.im_hi, out_J.im_lo};
    int64_t max_m = 0;
    for (int p = 0; p < S->n_polys; ++p)
        max_m = std::max<int64_t>(max_m, S->poly_start[p + 1] - S->poly_start[p]);

    // time one candidate (pins it); < 0 if it does not fit
    struct Cand {
        int L, cc, nt, G, T, nbuf;
        float ms;
    };
    auto time_one = [&](Cand &c) -> pe_status {
        {
            std::lock_guard<std::mutex> lock(S->mu);
            S->pin_L = c.L;
            S->pin_cc = c.cc;
            S->pin_nt = c.nt;
            S->pin_G = c.G;
            S->pin_T = c.T;
            S->pin_nbuf = c.nbuf;
        }
        auto call = [&](hipStream_t ts) {
            std::lock_guard<std::mutex> lock(S->mu);
            return S->eval_locked(n_points, x, f, J, dd, ts, nullptr);
        };
        // calls per timed graph: about 20 ms of work, 1 to 10 calls
        float ms = 0.f;
        pe_status st = time_calls(hs, 1, call, ms);
        const int reps = ms > 0.f ? std::max(1, std::min(10, (int)(20.f / ms))) : 10;
        if (st == PE_OK && reps > 1) st = time_calls(hs, reps, call, ms);
        c.ms = st == PE_OK ? ms : -1.f;
        return st == PE_EUNSUPPORTED ? PE_OK : st;
    };
    auto unpin = [&] {
        std::lock_guard<std::mutex> lock(S->mu);
        S->pin_L = S->pin_cc = S->pin_nt = S->pin_G = S->pin_T = S->pin_nbuf = 0;
    };

    // stage 1: lanes, variables per lane, workgroup size and split, with
    // tiles of one point and one staging buffer
    std::vector<Cand> first;
    for (int cc : {2, 4, 8})
        for (int lm : {1, 2, 4}) {
            const int L = next_pow2(std::max(1, (std::max(1, S->max_k) + cc - 1) / cc)) * lm;
            if (L > 32) continue;
            for (int nt : {256, 512, 1024}) {
                const int MC = nt / L;
                if (MC < 1) continue;
                const int chunks = (int)std::max<int64_t>(1, (max_m + MC - 1) / MC);
                for (int G : {1, 2, 4}) {
                    if (G > chunks) continue;
                    if (G > 1 && n_points * S->n_polys >= 1024) continue;
                    Cand c{L, cc, nt, G, 1, 1, -1.f};
                    pe_status st = time_one(c);
                    if (st != PE_OK) {
                        unpin();
                        return st;
                    }
                    if (c.ms >= 0.f) first.push_back(c);
                }
            }
        }
    if (first.empty()) {
        unpin();
        return fail(PE_EUNSUPPORTED, "no schedule fits");
    }
    std::sort(first.begin(), first.end(), [](const Cand &a, const Cand &b) { return a.ms < b.ms; });
    Cand best = first[0];
    // stage 2: tiles of 2 to 8 points and two staging buffers, for the three
    // fastest schedules of stage 1 (the tile shape does not change the tables)
    const size_t top = std::min<size_t>(3, first.size());
    for (size_t i = 0; i < top; ++i)
        for (int T : {1, 2, 4, 8}) {
            if (T > n_points) continue;
            for (int nbuf : {1, 2}) {
                if (T == 1 && nbuf == 1) continue;
                Cand c = first[i];
                c.T = T;
                c.nbuf = nbuf;
                pe_status st = time_one(c);
                if (st != PE_OK) {
                    unpin();
                    return st;
                }
                if (c.ms >= 0.f && c.ms < best.ms) best = c;
            }
        }
    cache_store(cache_path, key, {best.L, best.cc, best.nt, best.G, best.T, best.nbuf});
    return pe_set_schedule(sys, best.L, best.cc, best.nt, best.G, best.T, best.nbuf);
}

}  // extern "C"
