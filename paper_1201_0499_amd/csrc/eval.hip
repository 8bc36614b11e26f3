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
//  3. Summation (Section 3.3) without the zero-padded dense term array: each
//     term is written to an LDS staging slot chosen on the host so that the
//     terms of one output are contiguous and in monomial order; the lanes
//     then add fixed-length pieces of those runs, and the first piece of each
//     output adds the piece sums of its output (kept in place of each
//     piece's first term) into an LDS accumulator.  All
//     orders are fixed by the host tables, so results are deterministic.
//
// With G > 1 the workgroups of one polynomial each write their partial row
// to global memory; the last to arrive (an integer ticket) adds the G
// partial rows in a fixed order and writes the result.
#include "dd.hpp"
#include "eval.hpp"
#include "monomial.hpp"
#include "device.hpp"
#include "newton.hpp"

namespace pe {

// Reads the lane's variables from the LDS power table (row 0 = x).
template <class C, int CC>
struct LdsX {
    const C *pw;
    int pos[CC];
    __device__ __forceinline__ C operator()(int t) const { return pw[pos[t]]; }
};

template <class A, int CC, int MAXT>
__global__ __launch_bounds__(MAXT) void eval_kernel(const EvalArgs a)
{
    using C = typename A::C;
    using IO = Io<A>;
    HIP_DYNAMIC_SHARED(double, lds_raw)
    __shared__ int s_last;

    const int n = a.n_vars;
    const int np1 = n + 1;
    const int NT = blockDim.x;
    const int tid = threadIdx.x;
    C *pw = reinterpret_cast<C *>(lds_raw);   // [R][np1]
    C *stage = pw + (size_t)a.R * np1;         // [stage_slots]
    C *acc = stage + a.stage_slots;            // [np1]
    const int trash = a.stage_slots - 1;

    const int q = tid & (a.L - 1);
    const int sl = tid >> a.log2L;
    const int group = blockIdx.x;
    const int p = group / a.G;
    const int c_begin = a.group_chunk0[group];
    const int c_end = a.group_chunk0[group + 1];
    const LaneGroup grp{a.L};

    for (int64_t pt = blockIdx.y; pt < a.n_points; pt += gridDim.y) {
        if (a.mask && a.mask[pt] != kRunning) continue;
        __syncthreads();
        // ---- stage 1: power table of the point (Section 3.1) ----
        for (int i = tid; i < n; i += NT) {
            const C x = IO::load(a.x, pt * n + i);
            pw[i] = x;
            C xr = x;
            for (int r = 1; r < a.R; ++r) {
                xr = A::mul(xr, x);
                pw[(size_t)r * np1 + i] = xr;
            }
        }
        for (int r = tid; r < a.R; r += NT) pw[(size_t)r * np1 + n] = A::one();
        for (int o = tid; o < np1; o += NT) acc[o] = A::zero();
        __syncthreads();

        for (int c = c_begin; c < c_end; ++c) {
            // chunk metadata and this lane's tables, loaded together
            const int4 ci = a.chunk_info[c];
            const int nm = ci.y & 0xFFFF;
            const int vbase = ci.y >> 16;
            const int pc0 = ci.z;
            const int npc = ci.w & 0xFFFF;
            const int PL = ci.w >> 16;
            const uint16_t *pst = a.piece_start + pc0 + c;
            const uint32_t *pout = a.piece_out + pc0;
            const bool active = sl < nm;
            const int64_t s = (int64_t)ci.x + (active ? sl : 0);
            LdsX<C, CC> xs{pw, {}};
            uint32_t wv[CC];
            int dst[CC];
            C coef = A::zero();
            if (active) {
                const uint32_t *wp = a.word + s * a.KP + q * CC;
                const uint16_t *dp = a.dest + s * a.KP + q * CC;
#pragma unroll
                for (int t = 0; t < CC; ++t) {
                    wv[t] = wp[t];
                    dst[t] = dp[t];
                }
                coef = IO::coef(a.coef, s);
            } else {
#pragma unroll
                for (int t = 0; t < CC; ++t) {
                    wv[t] = (uint32_t)n;  // dummy variable: value 1
                    dst[t] = trash;
                }
            }
            // this lane's first piece
            int my_b = 0, my_e = 0;
            uint32_t my_po = 0;
            if (tid < npc) {
                my_b = pst[tid];
                my_e = pst[tid + 1];
                my_po = pout[tid];
            }

            // ---- stage 2: monomials and their derivatives (Section 3.2) ----
            double ae[CC];
            C cf;
#pragma unroll
            for (int t = 0; t < CC; ++t) {
                const int pos = (int)(wv[t] & kPosMask);
                const int em1 = (int)(wv[t] >> kExpShift);
                xs.pos[t] = pos;
                ae[t] = (double)(em1 + 1);
                const int zrow = em1 > 0 ? em1 - 1 : 0;
                C z = pw[(size_t)zrow * np1 + pos];
                if (em1 == 0) z = A::one();
                cf = (t == 0) ? z : A::mul(cf, z);
            }
            C D[CC], V;
            monomial_terms<A, CC>(xs, cf, ae, coef, grp, D, V);
#pragma unroll
            for (int t = 0; t < CC; ++t) stage[dst[t]] = D[t];
            // value terms: butterfly sum over the groups of the wave (lanes
            // with the same q), so one slot per wave holds its monomials' sum
            if (!active) V = A::zero();
            for (int d = a.L; d < 64; d <<= 1) V = A::add(V, shfl_xor_c(V, d));
            if ((tid & 63) == 0) stage[vbase + (tid >> 6)] = V;
            __syncthreads();

            // ---- stage 3: summation (Section 3.3) ----
            // pieces: the sum of a piece replaces its first term
            for (int l = tid; l < npc; l += NT) {
                int b = my_b, e = my_e;
                if (l != tid) {
                    b = pst[l];
                    e = pst[l + 1];
                }
                if (e - b > 1) {
                    C sum = stage[b];
                    for (int j = b + 1; j < e; ++j) sum = A::add(sum, stage[j]);
                    stage[b] = sum;
                }
            }
            __syncthreads();
            // runs: the first piece of each output adds its run's pieces
            for (int l = tid; l < npc; l += NT) {
                int b = my_b;
                uint32_t po = my_po;
                if (l != tid) {
                    b = pst[l];
                    po = pout[l];
                }
                const int nrun = (int)(po >> kRunShift);
                if (nrun) {
                    const int o = (int)(po & kOutMask);
                    C sum = stage[b];
                    for (int j = 1; j < nrun; ++j) sum = A::add(sum, stage[b + j * PL]);
                    acc[o] = A::add(acc[o], sum);
                }
            }
            __syncthreads();
        }

        // ---- outputs: f_p and column p of J ----
        if (a.G == 1) {
            for (int o = tid; o < np1; o += NT) {
                const C v = acc[o];
                if (o == n)
                    IO::store(a.f, pt * a.n_polys + p, v);
                else if (a.J[0])
                    IO::store(a.J, pt * (int64_t)n * a.n_polys + (int64_t)o * a.n_polys + p, v);
            }
        } else {
            constexpr int W = A::kWords;
            double *mine = a.partial + ((pt * a.n_groups + group) * (int64_t)np1) * W;
            for (int o = tid; o < np1; o += NT) IO::put(mine + (int64_t)o * W, acc[o]);
            __syncthreads();  // every lane's partial stores precede the release below
            if (tid == 0) {
                __threadfence();  // release: partial row visible to the device
                const int t = atomicAdd(&a.tickets[pt * a.n_polys + p], 1);
                s_last = (t == a.G - 1);
                if (s_last) __threadfence();  // acquire the other groups' rows
            }
            __syncthreads();
            if (s_last) {
                const double *base = a.partial + ((pt * a.n_groups + (int64_t)p * a.G) * np1) * W;
                for (int o = tid; o < np1; o += NT) {
                    C v = IO::get(base + (int64_t)o * W);
                    for (int g = 1; g < a.G; ++g)
                        v = A::add(v, IO::get(base + ((int64_t)g * np1 + o) * W));
                    if (o == n)
                        IO::store(a.f, pt * a.n_polys + p, v);
                    else if (a.J[0])
                        IO::store(a.J, pt * (int64_t)n * a.n_polys + (int64_t)o * a.n_polys + p, v);
                }
                if (tid == 0) a.tickets[pt * a.n_polys + p] = 0;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------

using KernelFn = void (*)(const EvalArgs);

template <class A>
static KernelFn pick(int cc, int maxt)
{
#define PE_CASE(CCV, MT) \
    if (cc == CCV && maxt == MT) return eval_kernel<A, CCV, MT>;
    PE_CASE(2, 256) PE_CASE(2, 512) PE_CASE(2, 1024)
    PE_CASE(4, 256) PE_CASE(4, 512) PE_CASE(4, 1024)
    PE_CASE(8, 256) PE_CASE(8, 512) PE_CASE(8, 1024)
#undef PE_CASE
    return nullptr;
}

static KernelFn pick_any(int prec, int cc, int maxt)
{
    return prec == 1 ? pick<ArithDD>(cc, maxt) : pick<Arith64>(cc, maxt);
}

hipError_t launch_eval(int prec, int cc, int maxt, const EvalArgs &args, dim3 grid, dim3 block,
                       size_t lds_bytes, hipStream_t stream)
{
    KernelFn k = pick_any(prec, cc, maxt);
    if (!k) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, grid, block, lds_bytes, stream, args);
    return hipGetLastError();
}

hipError_t eval_kernels_init()
{
    const int ccs[3] = {2, 4, 8};
    const int mts[3] = {256, 512, 1024};
    for (int prec = 0; prec < 2; ++prec)
        for (int c : ccs)
            for (int m : mts) {
                KernelFn k = pick_any(prec, c, m);
                // best effort: a refusal shows up later as a launch error
                if (hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                        hipFuncAttributeMaxDynamicSharedMemorySize,
                                        160 * 1024) != hipSuccess)
                    (void)hipGetLastError();
            }
    return hipSuccess;
}

}  // namespace pe
