// Fused evaluation of a sparse polynomial system and its Jacobian on gfx950.
//
// One workgroup handles one polynomial (or a contiguous share of its
// monomials, when G > 1) at one point at a time.  The three stages of the
// paper (Section 2) run inside one kernel:
//
//  1. The point is read once, coalesced, and the power table x_i^r,
//     r = 1..R, of all variables is built in LDS by the lanes in parallel
//     (Section 3.1, first stage; R = d-1 for a maximal exponent d).  An
//     extra column holds the value 1 for padding entries.
//  2. Each monomial is handled by a group of L lanes, CC variables per lane:
//     common factor from the power table, Speelpenning partials with forward
//     and backward products in registers, coefficient and exponent scaling
//     (Sections 3.1 and 3.2; see monomial.hpp).  Supports, exponents and
//     coefficients are read coalesced: lane q of a group reads variables
//     q*CC .. q*CC+CC-1 of its monomial from a monomial-major table.
//  3. Summation (Section 3.3) without the zero-padded dense term array: the
//     outputs of a chunk are ranked by the length of their runs of terms;
//     row i of the LDS staging area holds the i-th term (in monomial
//     order) of every output with more than i terms, the j-th ranked
//     output's at slot rows[i] + j (slots chosen on the host).  The run of
//     rank j is added by 2^log2S lanes (as many as fit one round, up to 16;
//     one lane for large n), each with a cascaded accumulator over every
//     2^log2S-th row, then a butterfly over those lanes, and goes into the
//     output's LDS accumulator: the paper's one thread per output, per
//     chunk.  At each step consecutive lanes read consecutive slots, so the
//     reads are free of bank conflicts.  All orders are fixed, so results
//     are deterministic.
//
// A workgroup may also take a tile of T consecutive points (TILE = true,
// see eval_tile): the chunk inputs then serve all T points, whose power
// tables and accumulators sit side by side in LDS, and with two staging
// buffers one barrier per (chunk, point) item suffices.  Tiles of one point
// with one buffer run the one-point body (eval_group), whose code is free of
// the tile bookkeeping.
//
// With G > 1 the workgroups of one polynomial each write their partial row
// to global memory and a second small kernel (combine_kernel) adds the G
// rows in a fixed order; the kernel boundary makes the rows visible, so no
// device-wide fence is needed inside the evaluation.
//
// A second kernel runs many systems of different shapes in one persistent
// launch over a host-built task list (see batch_kernel).
#include <algorithm>
#include <atomic>
#include <mutex>

#include "dd.hpp"
#include "eval.hpp"
#include "monomial.hpp"
#include "device.hpp"

namespace pe {

// The lane's variables, held in registers, and their exponents, from the
// packed words.
template <class C, int CC>
struct RegX {
    C v[CC];
    __device__ __forceinline__ C operator()(int t) const { return v[t]; }
};

template <int CC>
struct WordExps {
    const uint32_t *wv;
    __device__ __forceinline__ double operator()(int t) const
    {
        return (double)((wv[t] >> kExpShift) + 1);
    }
};

// LDS carve-up of one workgroup for one system and a tile of T points (32
// bytes per complex double-double entry, 16 per complex FP64 one).
template <class A>
struct LdsLayout {
    LdsVec<A> pw;     // [T][R][n+1] power tables, column n = 1
    LdsVec<A> stage;  // [nbuf][stage_slots] term staging, last slot of each discards
    LdsVec<A> acc;    // [T][n+1] accumulators: J column entries, then f
    int *rows;        // [nbuf][max_rows+1] row starts of the staging area
};

// TILE = false: the one-point layout (T = 1, nbuf = 1, whatever the
// arguments say), with no run-time multiples in the offsets.
template <class A, bool TILE = true>
__device__ __forceinline__ LdsLayout<A> lds_layout(double2 *raw, const EvalArgs &a)
{
    const int T = TILE ? a.T : 1, nbuf = TILE ? a.nbuf : 1;
    LdsLayout<A> l;
    double2 *p = raw;
    l.pw = LdsVec<A>::at(p, T * a.R * (a.n_vars + 1), p);
    l.stage = LdsVec<A>::at(p, nbuf * a.stage_slots, p);
    l.acc = LdsVec<A>::at(p, T * (a.n_vars + 1), p);
    l.rows = reinterpret_cast<int *>(p);
    return l;
}

// Stage 1 (Section 3.1): the power table x_i^r, r = 1..R, of point pt, at
// entry `off` of the tables.  With x0 given, it is entry tid of the point
// (loaded by the caller, early); other entries are loaded here.
template <class A>
__device__ __forceinline__ void build_power_table(const EvalArgs &a, int64_t pt,
                                                  const LdsVec<A> &pw, int off,
                                                  const typename A::C *x0)
{
    using C = typename A::C;
    const int n = a.n_vars, np1 = n + 1, NT = blockDim.x, tid = threadIdx.x;
    for (int i = tid; i < n; i += NT) {
        const C x = (x0 && i == tid) ? *x0 : Io<A>::load(a.x, pt * n + i);
        pw.put(off + i, x);
        C xr = x;
        for (int r = 1; r < a.R; ++r) {
            xr = A::mul(xr, x);
            pw.put(off + r * np1 + i, xr);
        }
    }
    for (int r = tid; r < a.R; r += NT) pw.put(off + r * np1 + n, A::one());
}

// A lane's global inputs for one chunk: the chunk's header, its packed
// variables, the staging slots of its terms and the monomial's coefficient.
template <class A, int CC>
struct ChunkIn {
    int4 ci;  // first monomial, monomials | rows << 16, first row_start entry,
              // chunk index
    uint32_t wv[CC];
    uint32_t dv[CC / 2];  // slots of the lane's derivative terms, two per word
    uint32_t vd;          // slot of the monomial's value term
    typename A::C coef;
};

// The lane's first run of a chunk (output | run length << 16, by rank:
// lane t takes rank t >> log2S), fetched ahead; its later ranks are
// requested when the chunk starts.
using RunIn = uint32_t;

// rounds of ranks per lane whose run entries are requested together
constexpr int kRunRounds = 3;

// The lane's packed variables and coefficient for the chunk whose header is
// in.ci.
template <class A, int CC>
__device__ __forceinline__ void load_lane_in(const EvalArgs &a, ChunkIn<A, CC> &in)
{
    const int q = threadIdx.x & (a.L - 1);
    const int sl = threadIdx.x >> a.log2L;
    if (sl < (in.ci.y & 0xFFFF)) {
        const int64_t s = (int64_t)in.ci.x + sl;
        const uint32_t *wp = a.word + s * a.KP + q * CC;
        // CC is even, so the lane's CC slots start at an even index
        const uint32_t *dp = reinterpret_cast<const uint32_t *>(a.dest + s * a.KP + q * CC);
#pragma unroll
        for (int t = 0; t < CC; ++t) in.wv[t] = wp[t];
#pragma unroll
        for (int t = 0; t < CC / 2; ++t) in.dv[t] = dp[t];
        in.vd = a.vdest[s];
        in.coef = Io<A>::coef(a.coef, s);
    } else {
        in.vd = 0;
#pragma unroll
        for (int t = 0; t < CC; ++t) in.wv[t] = (uint32_t)a.n_vars;  // dummy variable: 1
#pragma unroll
        for (int t = 0; t < CC / 2; ++t) in.dv[t] = 0;
        in.coef = A::zero();
    }
}

template <class A, int CC>
__device__ __forceinline__ void load_chunk_in(const EvalArgs &a, int c, ChunkIn<A, CC> &in)
{
    in.ci = a.chunk_info[c];
    load_lane_in<A, CC>(a, in);
}

__device__ __forceinline__ RunIn load_run_in(const EvalArgs &a, const int4 &ci)
{
    const int j = (int)threadIdx.x >> a.log2S;
    return j <= a.n_vars ? a.run_info[(int64_t)ci.w * (a.n_vars + 1) + j] : 0u;
}

// Stages 2 and 3 for workgroup share `group` (polynomial group / G) at point
// pt.  On entry the power table of pt is in LDS, the accumulators are zero
// and in/rin hold the inputs of the group's first chunk; the inputs of each
// next chunk are fetched while the current one is being summed.  Ends with
// the outputs written (G == 1) or the partial row combined (G > 1).
template <class A, int CC, bool kGatherAhead>
__device__ __forceinline__ void eval_group(const EvalArgs &a, int group, int c_begin, int c_end,
                                           int64_t pt, const LdsLayout<A> &lds,
                                           ChunkIn<A, CC> &in, RunIn &rin)
{
    using C = typename A::C;
    using IO = Io<A>;
    const int n = a.n_vars;
    const int np1 = n + 1;
    const int NT = blockDim.x;
    const int tid = threadIdx.x;
    const LdsVec<A> &pw = lds.pw;
    const LdsVec<A> &stage = lds.stage;
    const LdsVec<A> &acc = lds.acc;
    const int q = tid & (a.L - 1);
    const int sl = tid >> a.log2L;
    const int p = group / a.G;
    const LaneGroup grp{a.L};

    // the lane's variables of a chunk, gathered from the power table into
    // registers, and their common-factor entries x^(a-1): row a-2 of the
    // table for a >= 2, and for a = 1 the padding column n, which holds 1 in
    // every row (an unconditional read instead of a select).  The table is
    // fixed for the point, so with kGatherAhead the next chunk's are
    // gathered while this one's summation ends, not by every wave at once
    // after the barrier.  The one-system kernel does so with up to four
    // variables per lane; with eight, and in the batch kernel, the registers
    // held across the barrier cost more than the gathers.
    RegX<C, CC> xs;
    C cf;
    auto gather = [&]() {
#pragma unroll
        for (int t = 0; t < CC; ++t) {
            const int pos = (int)(in.wv[t] & kPosMask);
            const int em1 = (int)(in.wv[t] >> kExpShift);
            xs.v[t] = pw.get(pos);
            const C z = pw.get(em1 == 0 ? n : (em1 - 1) * np1 + pos);
            cf = (t == 0) ? z : A::mul(cf, z);
        }
    };
    for (int c = c_begin; c < c_end; ++c) {
        const int4 ci = in.ci;
        const int nm = ci.y & 0xFFFF, nrows = (int)((uint32_t)ci.y >> 16);
        const bool active = sl < nm;
        // the chunk's row starts, requested now and stored to LDS before the
        // staging barrier (the previous chunk is done with them)
        const int row_v = tid <= nrows ? (int)a.row_start[ci.z + tid] : 0;

        // ---- stage 2: monomials and their derivatives (Section 3.2) ----
        if (!kGatherAhead || c == c_begin) gather();
        const WordExps<CC> ae{in.wv};
        C D[CC], V;
        monomial_terms<A, CC>(xs, cf, ae, in.coef, grp, D, V);
        // values: added over groups of 2^log2VG monomials inside the wave
        // (inactive lanes hold 0), one staged term per group
        for (int d = a.L; d < (a.L << a.log2VG); d <<= 1) V = sum_xor_c<A>(V, d);
        if (active) {
#pragma unroll
            for (int t = 0; t < CC; ++t) stage.put((in.dv[t >> 1] >> (16 * (t & 1))) & 0xFFFFu, D[t]);
            if (q == 0 && (sl & ((1 << a.log2VG) - 1)) == 0) stage.put(in.vd, V);
        }
        for (int i = tid; i <= nrows; i += NT) lds.rows[i] = i == tid ? row_v : (int)a.row_start[ci.z + i];
        __syncthreads();

        // the next chunk's inputs, fetched while this one is summed
        if (c + 1 < c_end) load_chunk_in<A, CC>(a, c + 1, in);

        // ---- stage 3: summation (Section 3.3) ----
        // 2^log2S lanes per run: lane t takes rank j = t >> log2S in the
        // first round (see rank_in for further rounds) and rows i = sub,
        // sub + 2^log2S, ... of its run, at slots rows[i] + j; the parts are
        // combined with a butterfly
        const int *rows = lds.rows;
        const uint32_t *rinfo = a.run_info + (int64_t)ci.w * (n + 1);
        const int S = 1 << a.log2S;
        const int sub = tid & (S - 1);
        const int opr = NT >> a.log2S;  // ranks per round
        const int j_lane = tid >> a.log2S;
        // rank of the lane in round k: serpentine order (reversed in odd
        // rounds), so that the lanes with the longest runs of one round get
        // the shortest of the next; a last round with few ranks then falls
        // on the waves that finished first
        auto rank_in = [&](int k) { return k * opr + ((k & 1) ? opr - 1 - j_lane : j_lane); };
        uint32_t run_k[kRunRounds - 1];
#pragma unroll
        for (int k = 1; k < kRunRounds; ++k) {
            const int j = rank_in(k);
            run_k[k - 1] = j <= n ? rinfo[j] : 0u;
        }
        // the lane's rows of a run: blocks of at most kRunBlock of them,
        // even and odd ones in two cascaded accumulators (two reads in
        // flight), block sums added with the sloppy sum
        auto part_sum = [&](int j, int len) -> C {
            C total = A::zero();
            for (int i0 = sub; i0 < len; i0 += kRunBlock * S) {
                const int iend = min(len, i0 + kRunBlock * S);
                typename A::Acc s0 = A::acc(stage.get(rows[i0] + j));
                const C x1 = stage.get(rows[min(i0 + S, iend - 1)] + j);
                typename A::Acc s1 = A::acc(i0 + S < iend ? x1 : A::zero());
                int i = i0 + 2 * S;
                for (; i + S < iend; i += 2 * S) {
                    A::acc_add(s0, stage.get(rows[i] + j));
                    A::acc_add(s1, stage.get(rows[i + S] + j));
                }
                if (i < iend) A::acc_add(s0, stage.get(rows[i] + j));
                const C v = A::sum(A::acc_get(s0), A::acc_get(s1));
                total = i0 == sub ? v : A::sum(total, v);
            }
            return total;
        };
        // one round: every lane takes part (ranks past the last output and
        // rows past a run's end give 0), so the butterfly runs with all lanes
        auto round = [&](int j, uint32_t ri) {
            const int len = j <= n ? (int)(ri >> 16) : 0;
            C v = part_sum(j, len);
            for (int d = 1; d < S; d <<= 1) v = sum_xor_c<A>(v, d);
            if (sub == 0 && len > 0) {
                const int o = (int)(ri & 0xFFFFu);
                acc.put(o, A::sum(acc.get(o), v));
            }
        };
        round(j_lane, rin);
#pragma unroll
        for (int k = 1; k < kRunRounds; ++k)
            if (k * opr <= n) round(rank_in(k), run_k[k - 1]);
        for (int k = kRunRounds; k * opr <= n; ++k) {
            const int j = rank_in(k);
            round(j, j <= n ? rinfo[j] : 0u);
        }
        if (c + 1 < c_end) {
            rin = load_run_in(a, in.ci);
            if (kGatherAhead) gather();
        }
        __syncthreads();
    }

    // ---- outputs: f_p and column p of J ----
    if (a.G == 1) {
        for (int o = tid; o < np1; o += NT) {
            const C v = acc.get(o);
            if (o == n)
                IO::store(a.f, pt * a.n_polys + p, v);
            else if (a.J[0])
                IO::store(a.J, pt * (int64_t)n * a.n_polys + (int64_t)o * a.n_polys + p, v);
        }
    } else {
        // partial row of this share, entry (o, p) of its group's block
        // [o][n_polys] (so combine_kernel reads consecutive p coalesced;
        // neighbouring polynomials run on one XCD, whose L2 merges the lines)
        constexpr int W = A::kWords;
        const int g = group - p * a.G;
        double *blk = a.partial + (pt * a.G + g) * (int64_t)np1 * a.n_polys * W;
        for (int o = tid; o < np1; o += NT)
            IO::put(blk + ((int64_t)o * a.n_polys + p) * W, acc.get(o));
    }
}

// Stages 2 and 3 for workgroup share `group` (polynomial group / G) at the
// tile of points pt0 .. pt0+npt-1, of which those with their bit set in
// `live` are evaluated.  On entry the tile's power tables are in LDS, its
// accumulators are initialised and in/rin hold the inputs of the group's
// first chunk.
//
// The work is a sequence of items (chunk, point), chunk-major: a chunk's
// inputs, read once from global memory, serve every point of the tile, and
// the inputs of the next chunk are fetched while the last point of the
// current one is summed.  Each item computes its monomials' terms into a
// staging buffer, waits at a barrier, and adds the buffer's runs into its
// point's accumulators.  With two staging buffers (nbuf = 2) an item's terms
// go to the buffer the previous item is not reading, so one barrier per
// item suffices: a lane that has summed item i and computes item i+1 writes
// the other buffer, and item i+2, which reuses this one, starts only after
// the barrier of item i+1, which every lane reaches after summing item i.
// Ends with the outputs written (G == 1) or the partial rows written
// (G > 1).
template <class A, int CC>
__device__ __forceinline__ void eval_tile(const EvalArgs &a, int group, int c_begin, int c_end,
                                          int64_t pt0, int npt, uint32_t live,
                                          const LdsLayout<A> &lds, ChunkIn<A, CC> &in,
                                          RunIn &rin)
{
    using C = typename A::C;
    using IO = Io<A>;
    const int n = a.n_vars;
    const int np1 = n + 1;
    const int NT = blockDim.x;
    const int tid = threadIdx.x;
    const LdsVec<A> &pw = lds.pw;
    const LdsVec<A> &stage = lds.stage;
    const LdsVec<A> &acc = lds.acc;
    const int q = tid & (a.L - 1);
    const int sl = tid >> a.log2L;
    const int p = group / a.G;
    const LaneGroup grp{a.L};
    const int PW = a.R * np1;          // power-table entries of one point
    const int RS = a.max_rows + 1;     // row-table entries of one staging buffer
    const int last_t = 31 - __clz(live);
    int b = 0;                         // staging buffer of the current item

    // summation geometry: 2^log2S lanes per run; lane t takes rank
    // j = t >> log2S in the first round (see rank_in for further rounds) and
    // rows i = sub, sub + 2^log2S, ... of its run, at slots rows[i] + j; the
    // parts are combined with a butterfly
    const int S = 1 << a.log2S;
    const int sub = tid & (S - 1);
    const int opr = NT >> a.log2S;  // ranks per round
    const int j_lane = tid >> a.log2S;
    // rank of the lane in round k: serpentine order (reversed in odd
    // rounds), so that the lanes with the longest runs of one round get
    // the shortest of the next; a last round with few ranks then falls
    // on the waves that finished first
    auto rank_in = [&](int k) { return k * opr + ((k & 1) ? opr - 1 - j_lane : j_lane); };

    for (int c = c_begin; c < c_end; ++c) {
        const int4 ci = in.ci;
        const int nm = ci.y & 0xFFFF, nrows = (int)((uint32_t)ci.y >> 16);
        const bool active = sl < nm;
        // the chunk's row starts, requested now and stored to LDS before each
        // item's staging barrier
        const int row_v = tid <= nrows ? (int)a.row_start[ci.z + tid] : 0;
        const uint32_t *rinfo = a.run_info + (int64_t)ci.w * (n + 1);
        uint32_t run_k[kRunRounds - 1];
#pragma unroll
        for (int k = 1; k < kRunRounds; ++k) {
            const int j = rank_in(k);
            run_k[k - 1] = j <= n ? rinfo[j] : 0u;
        }
        const RunIn rin_c = rin;

        for (int t = 0; t <= last_t; ++t) {
            if (!((live >> t) & 1u)) continue;
            const int pwo = t * PW;
            const int so = b * a.stage_slots;
            int *rows = lds.rows + b * RS;

            // ---- stage 2: monomials and their derivatives (Section 3.2) ----
            // the lane's variables and their common-factor entries, as in
            // eval_group, from the point's power table
            RegX<C, CC> xs;
            C cf;
#pragma unroll
            for (int u = 0; u < CC; ++u) {
                const int pos = (int)(in.wv[u] & kPosMask);
                const int em1 = (int)(in.wv[u] >> kExpShift);
                xs.v[u] = pw.get(pwo + pos);
                const C z = pw.get(pwo + (em1 == 0 ? n : (em1 - 1) * np1 + pos));
                cf = (u == 0) ? z : A::mul(cf, z);
            }
            const WordExps<CC> ae{in.wv};
            C D[CC], V;
            monomial_terms<A, CC>(xs, cf, ae, in.coef, grp, D, V);
            // values: added over groups of 2^log2VG monomials inside the wave
            // (inactive lanes hold 0), one staged term per group
            for (int d = a.L; d < (a.L << a.log2VG); d <<= 1) V = sum_xor_c<A>(V, d);
            if (active) {
#pragma unroll
                for (int u = 0; u < CC; ++u)
                    stage.put(so + (int)((in.dv[u >> 1] >> (16 * (u & 1))) & 0xFFFFu), D[u]);
                if (q == 0 && (sl & ((1 << a.log2VG) - 1)) == 0) stage.put(so + (int)in.vd, V);
            }
            for (int i = tid; i <= nrows; i += NT)
                rows[i] = i == tid ? row_v : (int)a.row_start[ci.z + i];
            __syncthreads();

            // the next chunk's inputs, fetched while the chunk's last item is
            // summed (no item of this chunk reads `in` after this point)
            const bool chunk_done = t == last_t;
            if (chunk_done && c + 1 < c_end) load_chunk_in<A, CC>(a, c + 1, in);

            // ---- stage 3: summation (Section 3.3) ----
            const int ao = t * np1;
            // the lane's rows of a run: blocks of at most kRunBlock of them,
            // even and odd ones in two cascaded accumulators (two reads in
            // flight), block sums added with the sloppy sum
            auto part_sum = [&](int j, int len) -> C {
                C total = A::zero();
                for (int i0 = sub; i0 < len; i0 += kRunBlock * S) {
                    const int iend = min(len, i0 + kRunBlock * S);
                    typename A::Acc s0 = A::acc(stage.get(so + rows[i0] + j));
                    const C x1 = stage.get(so + rows[min(i0 + S, iend - 1)] + j);
                    typename A::Acc s1 = A::acc(i0 + S < iend ? x1 : A::zero());
                    int i = i0 + 2 * S;
                    for (; i + S < iend; i += 2 * S) {
                        A::acc_add(s0, stage.get(so + rows[i] + j));
                        A::acc_add(s1, stage.get(so + rows[i + S] + j));
                    }
                    if (i < iend) A::acc_add(s0, stage.get(so + rows[i] + j));
                    const C v = A::sum(A::acc_get(s0), A::acc_get(s1));
                    total = i0 == sub ? v : A::sum(total, v);
                }
                return total;
            };
            // one round: every lane takes part (ranks past the last output and
            // rows past a run's end give 0), so the butterfly runs with all lanes
            auto round = [&](int j, uint32_t ri) {
                const int len = j <= n ? (int)(ri >> 16) : 0;
                C v = part_sum(j, len);
                for (int d = 1; d < S; d <<= 1) v = sum_xor_c<A>(v, d);
                if (sub == 0 && len > 0) {
                    const int o = ao + (int)(ri & 0xFFFFu);
                    acc.put(o, A::sum(acc.get(o), v));
                }
            };
            round(j_lane, rin_c);
#pragma unroll
            for (int k = 1; k < kRunRounds; ++k)
                if (k * opr <= n) round(rank_in(k), run_k[k - 1]);
            for (int k = kRunRounds; k * opr <= n; ++k) {
                const int j = rank_in(k);
                round(j, j <= n ? rinfo[j] : 0u);
            }
            if (chunk_done && c + 1 < c_end) rin = load_run_in(a, in.ci);
            if (a.nbuf > 1)
                b ^= 1;
            else
                __syncthreads();
        }
    }
    // with two buffers the last item's sums are complete only after a barrier
    if (a.nbuf > 1) __syncthreads();

    // ---- outputs: f_p and column p of J at every live point ----
    for (int t = 0; t <= last_t; ++t) {
        if (!((live >> t) & 1u)) continue;
        const int64_t pt = pt0 + t;
        const int ao = t * np1;
        if (a.G == 1) {
            for (int o = tid; o < np1; o += NT) {
                const C v = acc.get(ao + o);
                if (o == n)
                    IO::store(a.f, pt * a.n_polys + p, v);
                else if (a.J[0])
                    IO::store(a.J, pt * (int64_t)n * a.n_polys + (int64_t)o * a.n_polys + p, v);
            }
        } else {
            // partial row of this share, entry (o, p) of its group's block
            // [o][n_polys] (so combine_kernel reads consecutive p coalesced;
            // neighbouring polynomials run on one XCD, whose L2 merges the lines)
            constexpr int W = A::kWords;
            const int g = group - p * a.G;
            double *blk = a.partial + (pt * a.G + g) * (int64_t)np1 * a.n_polys * W;
            for (int o = tid; o < np1; o += NT)
                IO::put(blk + ((int64_t)o * a.n_polys + p) * W, acc.get(ao + o));
        }
    }
}

// The accumulators' initial values at entry `off`: zero, except the value
// output of a polynomial whose constant last monomial was folded, which
// starts at that coefficient.  `header` is the group's second header word:
// .z = index + 1 of the folded monomial (0: none); it is read only when the
// schedule folds some constant.
template <class A>
__device__ __forceinline__ void init_acc(const EvalArgs &a, const LdsLayout<A> &lds, int off,
                                         const int4 *header)
{
    for (int o = threadIdx.x; o <= a.n_vars; o += blockDim.x) lds.acc.put(off + o, A::zero());
    // the thread that zeroed the value output's entry overwrites it
    if (a.any_fold && (int)threadIdx.x == a.n_vars % (int)blockDim.x) {
        const int fold = header->z;
        if (fold > 0) lds.acc.put(off + a.n_vars, Io<A>::coef(a.coef, fold - 1));
    }
}

// Prepares the live points of the tile at pt0: their power tables and
// accumulators (callers add the barrier).  x0 is entry tid of point pt0 when
// tid < n, already loaded.  The tables come first: they depend on the points
// only, so they need not wait for anything the accumulators read.
template <class A>
__device__ __forceinline__ void begin_tile(const EvalArgs &a, int64_t pt0, uint32_t live,
                                           const LdsLayout<A> &lds,
                                           const typename A::C &x0, const int4 *header)
{
    const int PW = a.R * (a.n_vars + 1);
    for (int t = 0; t < 32 && (live >> t); ++t)
        if ((live >> t) & 1u) build_power_table<A>(a, pt0 + t, lds.pw, t * PW, t == 0 ? &x0 : nullptr);
    for (int t = 0; t < 32 && (live >> t); ++t)
        if ((live >> t) & 1u) init_acc<A>(a, lds, t * (a.n_vars + 1), header);
}

// Prepares point pt for the one-point path: its power table and the
// accumulators (callers add the barrier).  x0 is entry tid of the point when
// tid < n, already loaded.
template <class A>
__device__ __forceinline__ void begin_point(const EvalArgs &a, int64_t pt,
                                            const LdsLayout<A> &lds,
                                            const typename A::C &x0, const int4 *header)
{
    build_power_table<A>(a, pt, lds.pw, 0, &x0);
    init_acc<A>(a, lds, 0, header);
}

// Workgroups are handed to the 8 XCDs of the chip in turn (workgroup i to
// XCD i mod 8), and each XCD has its own L2.  This maps the workgroup index
// to the share it works on so that each XCD takes a contiguous range of
// shares: the polynomials whose output entries share cache lines (J is
// polynomial-minor) then write them through one L2.  A bijection of
// [0, count) for any count; the results do not depend on it.
__device__ __forceinline__ int xcd_order(int i, int count)
{
    constexpr int kXcds = 8;
    const int xcd = i % kXcds, slot = i / kXcds;
    const int q = count / kXcds, r = count % kXcds;
    return xcd * q + min(xcd, r) + slot;
}

// One system: workgroup (group, tile block); tiles of T consecutive points,
// strided by gridDim.y.  A group with a single chunk keeps its inputs in
// registers for all its tiles; otherwise the first chunk's inputs are
// fetched again per tile.  The first point's entries are requested first, so
// that their latency overlaps the dependent loads of the group header and the
// chunk inputs.  Waves per SIMD the evaluation kernel is compiled for: two
// for double-double and FP64 (so that two workgroups of 256 threads share a
// CU), one for quad-double, whose values take eight registers each.
template <class A>
constexpr int kWavesPerEu = 2;
template <>
constexpr int kWavesPerEu<ArithQD> = 1;

template <class A, int CC, int MAXT, bool TILE>
__global__ __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu(kWavesPerEu<A>))) void
eval_kernel(const EvalArgs a)
{
    if constexpr (!TILE) {
        using C = typename A::C;
        HIP_DYNAMIC_SHARED(double2, lds_raw)
        const LdsLayout<A> lds = lds_layout<A, false>(lds_raw, a);
        const int group = xcd_order(blockIdx.x, gridDim.x);
        const int64_t pt0 = blockIdx.y;
        const bool has_x = (int)threadIdx.x < a.n_vars;
        // the first point's entry is requested before the tables
        C x0 = A::zero();
        if (pt0 < a.n_points && has_x) x0 = Io<A>::load(a.x, pt0 * a.n_vars + threadIdx.x);
        const int4 g0 = a.group_info[2 * group];
        const int4 g1 = a.group_info[2 * group + 1];
        const int c_begin = g0.x, c_end = g0.y;
        const bool single = c_end - c_begin == 1;
        ChunkIn<A, CC> in;
        RunIn rin = 0u;
        bool loaded = false, first = true;
        for (int64_t pt = pt0; pt < a.n_points; pt += gridDim.y) {
            if (a.mask && a.mask[pt] != kMaskLive) continue;
            if (!first) __syncthreads();  // the previous point is done with LDS
            first = false;
            if (pt != pt0 && has_x) x0 = Io<A>::load(a.x, pt * a.n_vars + threadIdx.x);
            if (!loaded && c_begin < c_end) {
                in.ci = make_int4(g0.z, g0.w, g1.x, g1.y);
                load_lane_in<A, CC>(a, in);
                rin = load_run_in(a, in.ci);
                loaded = single;
            }
            begin_point<A>(a, pt, lds, x0, a.group_info + 2 * group + 1);
            __syncthreads();
            eval_group<A, CC, (CC <= 4)>(a, group, c_begin, c_end, pt, lds, in, rin);
        }
    } else {
        using C = typename A::C;
        HIP_DYNAMIC_SHARED(double2, lds_raw)
        const LdsLayout<A> lds = lds_layout<A>(lds_raw, a);
        const int group = xcd_order(blockIdx.x, gridDim.x);
        const int T = a.T;
        const int64_t n_tiles = (a.n_points + T - 1) / T;
        const int64_t tile0 = blockIdx.y;
        const bool has_x = (int)threadIdx.x < a.n_vars;
        // the first point's entry is requested before the tables
        C x0 = A::zero();
        if (tile0 < n_tiles && has_x) x0 = Io<A>::load(a.x, tile0 * T * a.n_vars + threadIdx.x);
        const int4 g0 = a.group_info[2 * group];
        const int4 g1 = a.group_info[2 * group + 1];
        const int c_begin = g0.x, c_end = g0.y;
        const bool single = c_end - c_begin == 1;
        ChunkIn<A, CC> in;
        RunIn rin = 0u;
        bool loaded = false, first = true;
        for (int64_t tile = tile0; tile < n_tiles; tile += gridDim.y) {
            const int64_t pt0 = tile * T;
            const int npt = (int)min<int64_t>(T, a.n_points - pt0);
            uint32_t live = npt >= 32 ? 0xFFFFFFFFu : ((1u << npt) - 1u);
            if (a.mask)
                for (int t = 0; t < npt; ++t)
                    if (a.mask[pt0 + t] != kMaskLive) live &= ~(1u << t);
            if (!live) continue;
            if (!first) __syncthreads();  // the previous tile is done with LDS
            first = false;
            if (tile != tile0 && has_x) x0 = Io<A>::load(a.x, pt0 * a.n_vars + threadIdx.x);
            if (!loaded && c_begin < c_end) {
                in.ci = make_int4(g0.z, g0.w, g1.x, g1.y);
                load_lane_in<A, CC>(a, in);
                rin = load_run_in(a, in.ci);
                loaded = single;
            }
            begin_tile<A>(a, pt0, live, lds, x0, a.group_info + 2 * group + 1);
            __syncthreads();
            eval_tile<A, CC>(a, group, c_begin, c_end, pt0, npt, live, lds, in, rin);
        }
    }
}

// Many systems in one persistent launch: workgroup b takes the tasks
// b, b + gridDim.x, ... of a host-ordered list (longest first); a task is one
// point of one system and a range of its polynomials, which share the power
// table built once for the task.
template <class A, int CC, int MAXT>
__global__ __launch_bounds__(MAXT) void batch_kernel(const BatchArgs b)
{
    using C = typename A::C;
    HIP_DYNAMIC_SHARED(double2, lds_raw)
    ChunkIn<A, CC> in;
    RunIn rin = 0u;
    for (int64_t t = blockIdx.x; t < b.n_tasks; t += gridDim.x) {
        const BatchTask task = b.tasks[t];
        const BatchDesc &d = b.desc[task.sys];
        EvalArgs a = d.a;
        for (int q = 0; q < 4; ++q) {
            a.x[q] = b.x[q] ? b.x[q] + d.x_off : nullptr;
            a.f[q] = b.f[q] ? b.f[q] + d.f_off : nullptr;
            a.J[q] = b.J[q] ? b.J[q] + d.J_off : nullptr;
        }
        const LdsLayout<A> lds = lds_layout<A, false>(lds_raw, a);
        __syncthreads();  // the previous task is done with LDS
        for (int p = task.p0; p < task.p1; ++p) {
            const int4 g0 = a.group_info[2 * p];
            const int4 g1 = a.group_info[2 * p + 1];
            if (g0.x < g0.y) {
                in.ci = make_int4(g0.z, g0.w, g1.x, g1.y);
                load_lane_in<A, CC>(a, in);
                rin = load_run_in(a, in.ci);
            }
            if (p == task.p0) {
                C x0 = A::zero();
                if ((int)threadIdx.x < a.n_vars)
                    x0 = Io<A>::load(a.x, task.pt * a.n_vars + threadIdx.x);
                begin_point<A>(a, task.pt, lds, x0, a.group_info + 2 * p + 1);
            } else {
                __syncthreads();  // the previous polynomial's outputs have been read
                init_acc<A>(a, lds, 0, a.group_info + 2 * p + 1);
            }
            __syncthreads();
            eval_group<A, CC, false>(a, p, g0.x, g0.y, task.pt, lds, in, rin);
        }
    }
}

// f and J from the G partial rows of each (point, polynomial), added in
// workgroup order.  Thread e of a point takes entry (o, p) with
// e = o * n_polys + p, so consecutive threads write consecutive entries of
// J (and of f, o = n_vars).  The host guarantees (n_vars+1)*n_polys < 2^31.
template <class A>
__global__ __launch_bounds__(256) void combine_kernel(const EvalArgs a)
{
    using C = typename A::C;
    using IO = Io<A>;
    constexpr int W = A::kWords;
    const int n = a.n_vars, np1 = n + 1, P = a.n_polys;
    const int total = np1 * P;
    const int stride = gridDim.x * blockDim.x;
    const int64_t blk = (int64_t)total * W;  // one group's block [o][n_polys]
    for (int64_t pt = blockIdx.y; pt < a.n_points; pt += gridDim.y) {
        if (a.mask && a.mask[pt] != kMaskLive) continue;
        const double *rows = a.partial + pt * a.G * blk;
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
            const int o = e / P, p = e - o * P;
            const double *src = rows + (int64_t)e * W;
            C v = IO::get(src);
            for (int g = 1; g < a.G; ++g) v = A::sum(v, IO::get(src + g * blk));
            if (o == n)
                IO::store(a.f, pt * P + p, v);
            else if (a.J[0])
                IO::store(a.J, pt * (int64_t)n * P + e, v);
        }
    }
}

hipError_t launch_combine(int prec, const EvalArgs &args, hipStream_t stream)
{
    const int64_t total = (int64_t)args.n_polys * (args.n_vars + 1);
    if (total <= 0 || args.n_points <= 0) return hipSuccess;
    const unsigned bx = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
    const unsigned by = (unsigned)std::min<int64_t>(args.n_points, 65535);
    if (prec == 2)
        hipLaunchKernelGGL(combine_kernel<ArithQD>, dim3(bx, by), dim3(256), 0, stream, args);
    else if (prec == 1)
        hipLaunchKernelGGL(combine_kernel<ArithDD>, dim3(bx, by), dim3(256), 0, stream, args);
    else
        hipLaunchKernelGGL(combine_kernel<Arith64>, dim3(bx, by), dim3(256), 0, stream, args);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------

using KernelFn = void (*)(const EvalArgs);

template <class A, bool TILE>
static KernelFn pick(int cc, int maxt)
{
#define PE_CASE(CCV, MT) \
    if (cc == CCV && maxt == MT) return eval_kernel<A, CCV, MT, TILE>;
    PE_CASE(2, 256) PE_CASE(2, 512) PE_CASE(2, 1024)
    PE_CASE(4, 256) PE_CASE(4, 512) PE_CASE(4, 1024)
    PE_CASE(8, 256) PE_CASE(8, 512) PE_CASE(8, 1024)
#undef PE_CASE
    return nullptr;
}

// quad-double: 256 threads with two or four variables per lane, or 512
// threads with two (two waves per SIMD); one point per workgroup
static KernelFn pick_qd(int cc, int maxt)
{
    if (maxt == 512) return cc == 2 ? eval_kernel<ArithQD, 2, 512, false> : nullptr;
    if (maxt != 256) return nullptr;
    if (cc == 2) return eval_kernel<ArithQD, 2, 256, false>;
    if (cc == 4) return eval_kernel<ArithQD, 4, 256, false>;
    return nullptr;
}

static KernelFn pick_any(int prec, int cc, int maxt, bool tile)
{
    if (prec == 2) return tile ? nullptr : pick_qd(cc, maxt);
    if (prec == 1) return tile ? pick<ArithDD, true>(cc, maxt) : pick<ArithDD, false>(cc, maxt);
    return tile ? pick<Arith64, true>(cc, maxt) : pick<Arith64, false>(cc, maxt);
}

// Tiles of one point with one staging buffer run the one-point kernel body;
// anything else the tiled one.
hipError_t launch_eval(int prec, int cc, int maxt, const EvalArgs &args, dim3 grid, dim3 block,
                       size_t lds_bytes, hipStream_t stream)
{
    KernelFn k = pick_any(prec, cc, maxt, args.T > 1 || args.nbuf > 1);
    if (!k) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, grid, block, lds_bytes, stream, args);
    return hipGetLastError();
}

using BatchFn = void (*)(const BatchArgs);

template <class A>
static BatchFn pick_batch(int cc, int maxt)
{
#define PE_CASE(CCV, MT) \
    if (cc == CCV && maxt == MT) return batch_kernel<A, CCV, MT>;
    PE_CASE(2, 256) PE_CASE(2, 512) PE_CASE(2, 1024)
    PE_CASE(4, 256) PE_CASE(4, 512) PE_CASE(4, 1024)
    PE_CASE(8, 256) PE_CASE(8, 512) PE_CASE(8, 1024)
#undef PE_CASE
    return nullptr;
}

hipError_t launch_batch(int prec, int cc, int maxt, const BatchArgs &args, dim3 grid, dim3 block,
                        size_t lds_bytes, hipStream_t stream)
{
    BatchFn k = prec == 1 ? pick_batch<ArithDD>(cc, maxt) : pick_batch<Arith64>(cc, maxt);
    if (!k) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, grid, block, lds_bytes, stream, args);
    return hipGetLastError();
}

int batch_occupancy(int prec, int cc, int maxt, int threads, size_t lds_bytes)
{
    BatchFn k = prec == 1 ? pick_batch<ArithDD>(cc, maxt) : pick_batch<Arith64>(cc, maxt);
    int blocks = 0;
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void *>(k),
                                                           threads, lds_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return blocks > 0 ? blocks : 1;
}

// The static scratch of the allocation-free evaluation.  In host code the
// name `scratch` is only a stand-in for the symbol: its device address, which
// differs per device, comes from hipGetSymbolAddress and is the only handle
// passed to kernels.
static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

constexpr int kMaxScratchDevices = 64;
static std::atomic<void *> g_scratch_ptr[kMaxScratchDevices];
static std::mutex g_scratch_mu;

hipError_t static_scratch_setup()
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev].load()) return hipSuccess;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev].store(p);
    return hipSuccess;
}

void *static_scratch_ptr(int device)
{
    if (device < 0 || device >= kMaxScratchDevices) return nullptr;
    return g_scratch_ptr[device].load();
}

hipError_t eval_kernels_init()
{
    const int ccs[3] = {2, 4, 8};
    const int mts[3] = {256, 512, 1024};
    for (int prec = 0; prec < 2; ++prec)
        for (int c : ccs)
            for (int m : mts) {
                const void *ks[3] = {reinterpret_cast<const void *>(pick_any(prec, c, m, false)),
                                     reinterpret_cast<const void *>(pick_any(prec, c, m, true)),
                                     reinterpret_cast<const void *>(
                                         prec == 1 ? pick_batch<ArithDD>(c, m)
                                                   : pick_batch<Arith64>(c, m))};
                // best effort: a refusal shows up later as a launch error
                for (const void *k : ks)
                    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            kMaxLds) != hipSuccess)
                        (void)hipGetLastError();
            }
    for (int c : {2, 4})
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(pick_qd(c, 256)),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds) != hipSuccess)
            (void)hipGetLastError();
    return hipSuccess;
}

}  // namespace pe
