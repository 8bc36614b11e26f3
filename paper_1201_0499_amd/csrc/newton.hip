// Kernels of the Newton corrector that consumes the evaluator (the paper's
// motivation: Newton's method inside path trackers, Section 1 and the
// abstract, where evaluating f and its Jacobian is the costly step).
//
//  resid      f(x) in complex double-double or quad-double, values only:
//             one workgroup per start builds the power table x_i^r,
//             r = 1..d, in LDS; each wave takes whole polynomials, its lanes
//             stride over the monomials (c * prod x^a from the table) and the
//             wave sums them with a butterfly.  Deterministic order.
//  check      residual norm max_p |f_p| and the per-start status.
//  lu_solve   J d = r by Gaussian elimination with partial pivoting, one
//             workgroup per start, J column-major in global memory, in
//             complex FP64 or complex dd (templated on the arithmetic).
//  gj_small, gj_panel
//             the FP64 solve for n <= 128 by Gauss-Jordan elimination with
//             partial pivoting, the matrix in registers of one workgroup.
//  update     x <- x - d in dd (or quad-double).
#include <type_traits>
#include <vector>

#include "dd.hpp"
#include "device.hpp"
#include "eval.hpp"
#include "newton.hpp"
#include "lds_budget.hpp"
#include "packing.hpp"

static_assert(pe::kRunning == pe::kMaskLive, "running starts are the evaluation's live points");

namespace pe {

// ---------------------------------------------------------------------------
// residual f(x), complex double-double
// ---------------------------------------------------------------------------

template <class A, int NT>
__global__ __launch_bounds__(NT) void resid_kernel(const ResidArgs a)
{
    using C = typename A::C;
    using IO = Io<A>;
    HIP_DYNAMIC_SHARED(double2, lds_raw)
    const int64_t pt = blockIdx.x;
    if (a.status && a.status[pt] != kRunning) return;
    const int n = a.n_vars;
    const int np1 = n + 1;
    const int tid = threadIdx.x;
    double2 *next = lds_raw;
    const LdsVec<A> pw = LdsVec<A>::at(lds_raw, a.R * np1, next);  // [R][np1]: x^1 .. x^R

    for (int i = tid; i < n; i += NT) {
        const C x = IO::load(a.x, pt * n + i);
        pw.put(i, x);
        C xr = x;
        for (int r = 1; r < a.R; ++r) {
            xr = A::mul(xr, x);
            pw.put(r * np1 + i, xr);
        }
    }
    __syncthreads();

    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int n_waves = NT >> 6;
    for (int p = wave; p < a.n_polys; p += n_waves) {
        C sum = A::zero();
        for (int64_t s = a.poly_start[p] + lane; s < a.poly_start[p + 1]; s += 64) {
            C v = IO::coef(a.coef, s);
            const int j1 = a.mono_start[s + 1];
            int j = a.mono_start[s];
            // four support words requested together, so that one memory
            // latency covers four factors instead of one
            for (; j + 4 <= j1; j += 4) {
                uint32_t w[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) w[t] = a.word[j + t];
                C g[4];
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    g[t] = pw.get((int)(w[t] >> kExpShift) * np1 + (int)(w[t] & kPosMask));
                v = A::mul(v, A::mul(A::mul(g[0], g[1]), A::mul(g[2], g[3])));
            }
            for (; j < j1; ++j) {
                const uint32_t w = a.word[j];
                v = A::mul(v, pw.get((int)(w >> kExpShift) * np1 + (int)(w & kPosMask)));
            }
            sum = A::sum(sum, v);
        }
        sum = sum_xor<A, 1>(sum);
        sum = sum_xor<A, 2>(sum);
        sum = sum_xor<A, 4>(sum);
        sum = sum_xor<A, 8>(sum);
        sum = sum_xor<A, 16>(sum);
        sum = sum_xor<A, 32>(sum);
        if (lane == 0) IO::store(a.f, pt * a.n_polys + p, sum);
    }
}

// Double-double: 16 waves share one power table, four per SIMD to hide the
// latency of the table gathers.  Quad-double: 8 waves, whose values need
// twice the registers.
constexpr int kResidThreads = 1024;
constexpr int kResidThreadsQD = 512;

static size_t resid_lds(int prec, int32_t n, int32_t R)
{
    const size_t w = prec == 2 ? sizeof(ArithQD::C) : sizeof(ArithDD::C);
    return w * (size_t)R * ((size_t)n + 1);
}

bool resid_fits(int prec, int32_t n, int32_t R) { return resid_lds(prec, n, R) <= kMaxLds; }

hipError_t launch_resid(const ResidArgs &a, int prec, hipStream_t stream)
{
    if (a.n_points <= 0) return hipSuccess;
    const size_t lds = resid_lds(prec, a.n_vars, a.R);
    if (prec == 2)
        hipLaunchKernelGGL((resid_kernel<ArithQD, kResidThreadsQD>), dim3((unsigned)a.n_points),
                           dim3(kResidThreadsQD), lds, stream, a);
    else
        hipLaunchKernelGGL((resid_kernel<ArithDD, kResidThreads>), dim3((unsigned)a.n_points),
                           dim3(kResidThreads), lds, stream, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// residual norm and status
// ---------------------------------------------------------------------------

__global__ void check_kernel(int64_t n_starts, int32_t n_polys, const double *f_re,
                             const double *f_im, double tol, int32_t max_iter, double *res,
                             const int32_t *iters, int32_t *status, int32_t *running)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_starts || status[s] != kRunning) return;
    double m = 0.0;
    bool finite = true;
    for (int p = 0; p < n_polys; ++p) {
        const double re = f_re[s * n_polys + p], im = f_im[s * n_polys + p];
        const double a = hypot(re, im);
        finite = finite && isfinite(a);
        m = fmax(m, a);
    }
    res[s] = finite ? m : __builtin_nan("");
    if (!finite)
        status[s] = 3;
    else if (m < tol)
        status[s] = 0;
    else if (iters[s] >= max_iter)
        status[s] = 1;
    else
        atomicAdd(running, 1);
}

hipError_t launch_check(int64_t n_starts, int32_t n_polys, const double *const f[4], double tol,
                        int32_t max_iter, double *res, const int32_t *iters, int32_t *status,
                        int32_t *running, hipStream_t stream)
{
    if (n_starts <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n_starts + 255) / 256);
    hipLaunchKernelGGL(check_kernel, dim3(blocks), dim3(256), 0, stream, n_starts, n_polys, f[0],
                       f[2], tol, max_iter, res, iters, status, running);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batched dense solve
// ---------------------------------------------------------------------------

template <class A>
struct Mat;

template <>
struct Mat<Arith64> {
    using C = Arith64::C;
    double *re, *im;
    __device__ __forceinline__ C get(int64_t i) const { return {re[i], im[i]}; }
    __device__ __forceinline__ void put(int64_t i, const C &v) const
    {
        re[i] = v.re;
        im[i] = v.im;
    }
};

template <>
struct Mat<ArithDD> {
    using C = ArithDD::C;
    double *rh, *rl, *ih, *il;
    __device__ __forceinline__ C get(int64_t i) const { return {{rh[i], rl[i]}, {ih[i], il[i]}}; }
    __device__ __forceinline__ void put(int64_t i, const C &v) const
    {
        rh[i] = v.re.hi;
        rl[i] = v.re.lo;
        ih[i] = v.im.hi;
        il[i] = v.im.lo;
    }
};

template <class A>
__device__ __forceinline__ Mat<A> make_mat(double *const (&p)[4], int64_t off);

template <>
__device__ __forceinline__ Mat<Arith64> make_mat<Arith64>(double *const (&p)[4], int64_t off)
{
    return {p[0] + off, p[2] + off};
}

template <>
__device__ __forceinline__ Mat<ArithDD> make_mat<ArithDD>(double *const (&p)[4], int64_t off)
{
    return {p[0] + off, p[1] + off, p[2] + off, p[3] + off};
}

// Value v of lane `src` (the same on every active lane) of the wave.
__device__ __forceinline__ double read_lane_d(double v, int src)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFll), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The same for the complex values of the two arithmetics.
__device__ __forceinline__ Arith64::C read_lane_c(const Arith64::C &v, int src)
{
    return {read_lane_d(v.re, src), read_lane_d(v.im, src)};
}

__device__ __forceinline__ ArithDD::C read_lane_c(const ArithDD::C &v, int src)
{
    return {{read_lane_d(v.re.hi, src), read_lane_d(v.re.lo, src)},
            {read_lane_d(v.im.hi, src), read_lane_d(v.im.lo, src)}};
}

// Value v of lane `src` (any lane of the wave, per lane) for the complex
// values of the two arithmetics.
__device__ __forceinline__ Arith64::C shfl_c(const Arith64::C &v, int src)
{
    return {__shfl(v.re, src, 64), __shfl(v.im, src, 64)};
}

__device__ __forceinline__ ArithDD::C shfl_c(const ArithDD::C &v, int src)
{
    return {{__shfl(v.re.hi, src, 64), __shfl(v.re.lo, src, 64)},
            {__shfl(v.im.hi, src, 64), __shfl(v.im.lo, src, 64)}};
}

// Larger maximum of a value over an aligned group of lanes (one butterfly
// step); the smaller of an index likewise.  DPP and row swaps, no LDS.
template <int OFF>
__device__ __forceinline__ double max_step(double v)
{
    const double o = xor_lane_d<OFF>(v);
    return o > v ? o : v;
}

template <int OFF>
__device__ __forceinline__ int min_step(int v)
{
    const int o = xor_lane_i<OFF>(v);
    return o < v ? o : v;
}

// One pass of a trailing update A -= L U over CB columns c0 .. c0+CB-1 of
// [J | d] (column n is the right-hand side; columns past ce are left alone)
// and R blocks of 64 rows from row `base` (rows from rend on are left
// alone): lane l takes rows base + l + 64 r.  L has nq <= NQ columns in LDS,
// L(i, q) at Lv[q ld + i - lrow0].  Entry e = q CB + b of u (lane e mod 64
// of register e / 64) holds -U(q, c0 + b) and reaches the whole wave through
// scalar registers when its turn comes.  All reads of the pass are issued
// before the arithmetic.  Every lane of the wave must take part (readlane).
template <class A, int NQ, int CB, int R>
__device__ __forceinline__ void trailing_pass(const Mat<A> &M, const Mat<A> &d,
                                              const LdsVec<A> &Lv, int ld, int lrow0, int nq,
                                              int n, int ce, int c0, int base, int rend,
                                              const typename A::C (&u)[(NQ * CB + 63) / 64])
{
    using C = typename A::C;
    const int i0 = base + (int)(threadIdx.x & 63);
    C acc[R][CB];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            const int c = c0 + b, i = i0 + 64 * r;
            acc[r][b] = i >= rend || c > ce ? A::zero()
                        : c < n             ? M.get((int64_t)c * n + i)
                                            : d.get(i);
        }
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        if (q < nq) {
            C l[R];
#pragma unroll
            for (int r = 0; r < R; ++r)
                l[r] = i0 + 64 * r < rend ? Lv.get(q * ld + (i0 + 64 * r - lrow0)) : A::zero();
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                const C ub = read_lane_c(u[(q * CB + b) / 64], (q * CB + b) % 64);
#pragma unroll
                for (int r = 0; r < R; ++r) acc[r][b] = A::add(acc[r][b], A::mul(l[r], ub));
            }
        }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            const int c = c0 + b, i = i0 + 64 * r;
            if (i < rend && c <= ce) {
                if (c < n)
                    M.put((int64_t)c * n + i, acc[r][b]);
                else
                    d.put(i, acc[r][b]);
            }
        }
}

// A -= L U over rows [rb, re) and columns [cb, ce] of [J | d], with L as in
// trailing_pass and U rows urow0 .. urow0+nq-1 of the same columns.  A wave
// takes CB columns at a time (their U entries one per lane and register), in
// passes of RB blocks of 64 rows.  FP64 then takes at most one pass each of 2 and 1
// blocks for what is left, so no pass computes a block wholly past the last
// row; double-double keeps one pass size (a second would give the kernel a
// private stack).  Trip counts are wave-uniform, as the readlanes require.
template <class A, int NQ, int CB, int RB, int NT>
__device__ __forceinline__ void trailing_update(const Mat<A> &M, const Mat<A> &d,
                                                const LdsVec<A> &Lv, int ld, int lrow0, int nq,
                                                int urow0, int n, int cb, int ce, int rb, int re)
{
    using C = typename A::C;
    constexpr int UL = (NQ * CB + 63) / 64;
    constexpr bool kF64 = sizeof(C) == 2 * sizeof(double);
    constexpr int n_waves = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c0 = cb + CB * wave; c0 <= ce; c0 += CB * n_waves) {
        C u_lane[UL];
#pragma unroll
        for (int g = 0; g < UL; ++g) {
            const int e = 64 * g + lane, q = e / CB, c = c0 + e - q * CB;
            u_lane[g] = q < nq && c <= ce ? A::neg(c < n ? M.get((int64_t)c * n + urow0 + q)
                                                         : d.get(urow0 + q))
                                          : A::zero();
        }
        int base = rb;
        if constexpr (kF64) {
            static_assert(!kF64 || RB == 4, "tail passes of 2 and 1 blocks");
            for (; base + 64 * (RB - 1) < re; base += 64 * RB)
                trailing_pass<A, NQ, CB, RB>(M, d, Lv, ld, lrow0, nq, n, ce, c0, base, re, u_lane);
            if (base + 64 < re) {
                trailing_pass<A, NQ, CB, 2>(M, d, Lv, ld, lrow0, nq, n, ce, c0, base, re, u_lane);
                base += 128;
            }
            if (base < re)
                trailing_pass<A, NQ, CB, 1>(M, d, Lv, ld, lrow0, nq, n, ce, c0, base, re, u_lane);
        } else {
            for (; base < re; base += 64 * RB)
                trailing_pass<A, NQ, CB, RB>(M, d, Lv, ld, lrow0, nq, n, ce, c0, base, re, u_lane);
        }
    }
}

// The row interchanges of the panel at rows jp .. jp+nbp-1 on columns
// [cb, ce] of [J | d]: cnt slots, row s_row[m] ends up with what slot
// s_from[m] held (slots 0 .. nbp-1 are the panel's top rows).  2 NB lanes
// per column, lane m with slot m: each lane reads its row, takes the value
// its row ends up with from the lane of its source slot and writes it back.
// With with_u the top rows instead compute U = L11^{-1} A by forward
// substitution across the lanes (row r subtracts L[r][q] u_q for q = 0, 1,
// ... in turn; L11 unit lower, from the panel in LDS) and write that.  A
// previous panel whose update of these columns is still pending (nqa > 0)
// is first applied to the top rows, as the trailing update would have:
// u -= La(jp + m, q) Ua(q, c) for q = 0, 1, ..., with La(jp + m, q) at
// las[m nqa + q] and Ua in rows ua0 .. ua0+nqa-1.  Trip counts are
// wave-uniform, as the shuffles require.
template <class A, int NB, int NT>
__device__ __forceinline__ void interchange(const Mat<A> &M, const Mat<A> &d,
                                            const LdsVec<A> &pan, int n, int jp, int nbp,
                                            int cnt, const int *s_row, const int *s_from, int cb,
                                            int ce, bool with_u, const LdsVec<A> &las, int nqa,
                                            int ua0)
{
    using C = typename A::C;
    constexpr int LPC = 2 * NB, CPW = 64 / LPC;
    static_assert(LPC <= 64 && 64 % LPC == 0, "columns tile the wave");
    constexpr int n_waves = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane % LPC, cw = lane / LPC;
    const int row = m < cnt ? s_row[m] : jp;
    const int src = cw * LPC + (m < cnt ? s_from[m] : m);
    for (int c0 = cb + CPW * wave; c0 <= ce; c0 += CPW * n_waves) {
        const int c = c0 + cw;
        const bool col = c <= ce;
        const Mat<A> &X = c < n ? M : d;
        const int64_t xc = c < n ? (int64_t)c * n : 0;
        C v = shfl_c(col && m < cnt ? X.get(xc + row) : A::zero(), src);
        if (col && m < cnt && (!with_u || m >= nbp)) X.put(xc + row, v);
        if (!with_u) continue;
        if (nqa > 0) {
            const C nua = col && m < nqa ? A::neg(X.get(xc + ua0 + m)) : A::zero();
            for (int q = 0; q < nqa; ++q) {
                const C ub = shfl_c(nua, cw * LPC + q);
                if (m < nbp) v = A::add(v, A::mul(las.get(m * nqa + q), ub));
            }
        }
        for (int q = 0; q + 1 < nbp; ++q) {
            const C uq = shfl_c(v, cw * LPC + q);
            if (m > q && m < nbp) v = A::add(v, A::mul(A::neg(pan.get(q * n + m)), uq));
        }
        if (col && m < nbp) X.put(xc + jp + m, v);
    }
}

// Blocked right-looking elimination with partial pivoting, one workgroup per
// start, the panels taken in pairs (A at columns j0.., B right of it):
//   1. a panel (rows jp..n-1) is copied to LDS and factored there, column
//      by column: pivot = largest |re|+|im| at or below the diagonal
//      (smallest row on ties; every thread reduces the waves' candidates
//      itself), row swap inside the panel, multipliers l = a / pivot,
//      rank-1 update of the panel's remaining columns;
//   2. the panel is written back, and its row swaps are turned into one
//      permutation of the rows they touch;
//   3. A: on the columns right of it and the right-hand side, which travels
//      along as column n, 2 NB lanes per column apply that permutation (one
//      read and one write per row, all in flight together) and compute
//      U_A = L11^{-1} A12 by forward substitution across the lanes; then
//      only panel B's columns get A's update A22 -= L21 U12;
//   4. B: factored like A; its permutation is applied to A's multipliers
//      and to the columns right of B, whose top rows also take A's update
//      before B's forward substitution;
//   5. the rows below both panels take both updates in one pass over the
//      trailing block, in row chunks whose multipliers (2 NB columns) are
//      staged in the LDS the panel used: the block is read and written once
//      per pair of panels.  Every element sees the same operations in the
//      same order as with one update per panel.
// Back substitution with U follows, column by column.
template <class A, int NB, int NT>
__global__ __launch_bounds__(NT) void lu_solve_kernel(int64_t n_starts, int32_t n, LuPlanes planes,
                                                      int32_t *status)
{
    using C = typename A::C;
    // narrow update (one panel): columns per wave, blocks of 64 rows per pass
    constexpr bool kF64 = sizeof(C) == 2 * sizeof(double);
    constexpr int CB = kF64 ? 4 : 2;
    constexpr int RB = kF64 ? 4 : 2;
    HIP_DYNAMIC_SHARED(double2, lds_raw)
    double2 *next = lds_raw;
    const LdsVec<A> pan = LdsVec<A>::at(lds_raw, NB * n, next);  // [NB][n]: column q, row r at q*n + r
    __shared__ double2 s_la_raw[NB * NB * (sizeof(C) / sizeof(double2))];
    double2 *next2 = s_la_raw;
    const LdsVec<A> las = LdsVec<A>::at(s_la_raw, NB * NB, next2);  // A's multipliers of B's top rows
    __shared__ double s_mag[NT / 64];
    __shared__ int s_idx[NT / 64];
    __shared__ int s_piv[NB];
    __shared__ int s_row[2 * NB], s_from[2 * NB], s_cnt;
    const int64_t st = blockIdx.x;
    if (status[st] != kRunning) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    constexpr int n_waves = NT / 64;
    const Mat<A> M = make_mat<A>(planes.J, st * (int64_t)n * n);
    const Mat<A> d = make_mat<A>(planes.d, st * (int64_t)n);
    // rows per chunk of the paired update: 2 NB multiplier columns in the
    // panel's LDS
    const int rch = max(1, (NB * n) / (2 * NB));

    // right-hand side: d = r (r is double-double; FP64 keeps the leading words)
    for (int i = tid; i < n; i += NT) {
        const int64_t k = st * (int64_t)n + i;
        if constexpr (sizeof(C) == 2 * sizeof(double))
            d.put(i, C{planes.r[0][k], planes.r[2][k]});
        else
            d.put(i, Io<ArithDD>::load(planes.r, k));
    }
    __syncthreads();
    bool bad = false;  // a zero or non-finite pivot: every thread sees the same

    for (int j0 = 0; j0 < n && !bad; j0 += 2 * NB) {
        const int nbA = min(NB, n - j0), jB = j0 + nbA;
        const int nbB = jB < n ? min(NB, n - jB) : 0, jC = jB + nbB;
        for (int h = 0; h < 2; ++h) {
            const int jp = h == 0 ? j0 : jB, nb = h == 0 ? nbA : nbB;
            if (nb == 0) break;
            const int rows = n - jp;
            // 1. panel to LDS and factor it
            for (int e = tid; e < rows * nb; e += NT) {
                const int q = e / rows, r = e - q * rows;
                pan.put(q * n + r, M.get((int64_t)(jp + q) * n + jp + r));
            }
            __syncthreads();
            for (int k = 0; k < nb; ++k) {
                double best = -1.0;
                int bi = n;
                for (int r = k + tid; r < rows; r += NT) {
                    const double mg = A::mag(pan.get(k * n + r));
                    if (mg > best || (mg == best && r < bi)) {
                        best = mg;
                        bi = r;
                    }
                }
                // the wave's largest magnitude, then the smallest row that
                // attains it (DPP and row swaps, no LDS round trips)
                double gm = best;
                gm = max_step<1>(gm);
                gm = max_step<2>(gm);
                gm = max_step<4>(gm);
                gm = max_step<8>(gm);
                gm = max_step<16>(gm);
                gm = max_step<32>(gm);
                int cand = best == gm ? bi : n;
                cand = min_step<1>(cand);
                cand = min_step<2>(cand);
                cand = min_step<4>(cand);
                cand = min_step<8>(cand);
                cand = min_step<16>(cand);
                cand = min_step<32>(cand);
                if (lane == 0) {
                    s_mag[wave] = gm;
                    s_idx[wave] = cand;
                }
                __syncthreads();
                // every thread reduces the waves' candidates itself, in one
                // order (the next writes to them come after two more barriers)
                double b = s_mag[0];
                int pr = s_idx[0];
                for (int w = 1; w < n_waves; ++w)
                    if (s_mag[w] > b || (s_mag[w] == b && s_idx[w] < pr)) {
                        b = s_mag[w];
                        pr = s_idx[w];
                    }
                if (!(b > 0.0) || !isfinite(b)) {
                    bad = true;
                    break;
                }
                if (tid == 0) s_piv[k] = pr;
                if (pr != k)
                    for (int q = tid; q < nb; q += NT) {
                        const C tk = pan.get(q * n + k), tp = pan.get(q * n + pr);
                        pan.put(q * n + k, tp);
                        pan.put(q * n + pr, tk);
                    }
                __syncthreads();
                const C inv = A::inv(pan.get(k * n + k));
                for (int r = k + 1 + tid; r < rows; r += NT) {
                    const C l = A::mul(pan.get(k * n + r), inv);
                    pan.put(k * n + r, l);
                    const C nl = A::neg(l);
                    for (int q = k + 1; q < nb; ++q)
                        pan.put(q * n + r,
                                A::add(pan.get(q * n + r), A::mul(nl, pan.get(q * n + k))));
                }
                __syncthreads();
            }
            if (bad) break;
            // 2. panel back to global memory; its interchanges as one
            // permutation of the rows they touch: the nb top rows (slots
            // 0 .. nb-1) and the distinct pivot rows below them
            for (int e = tid; e < rows * nb; e += NT) {
                const int q = e / rows, r = e - q * rows;
                M.put((int64_t)(jp + q) * n + jp + r, pan.get(q * n + r));
            }
            if (tid == 0) {
                int cnt = nb;
                for (int m = 0; m < nb; ++m) {
                    s_row[m] = jp + m;
                    s_from[m] = m;
                }
                for (int k = 0; k < nb; ++k) {
                    const int pr = jp + s_piv[k];
                    if (pr == jp + k) continue;
                    int sb = pr - jp;
                    if (sb >= nb) {
                        sb = -1;
                        for (int m = nb; m < cnt; ++m)
                            if (s_row[m] == pr) sb = m;
                        if (sb < 0) {
                            sb = cnt++;
                            s_row[sb] = pr;
                            s_from[sb] = sb;
                        }
                    }
                    const int t = s_from[k];
                    s_from[k] = s_from[sb];
                    s_from[sb] = t;
                }
                s_cnt = cnt;
            }
            __syncthreads();
            const int cnt = s_cnt;
            if (h == 0) {
                // 3. A's interchanges and U_A on every column right of it,
                // then A's update of panel B's columns only
                interchange<A, NB, NT>(M, d, pan, n, jp, nb, cnt, s_row, s_from, jB, n, true, las,
                                       0, 0);
                __syncthreads();
                if (nbB > 0) {
                    trailing_update<A, NB, CB, RB, NT>(M, d, pan, n, j0, nbA, j0, n, jB, jC - 1, jB,
                                                       n);
                    __syncthreads();
                }
            } else {
                // 4. B's interchanges on A's multipliers, then on the
                // columns right of B with A's update of their top rows
                interchange<A, NB, NT>(M, d, pan, n, jp, nb, cnt, s_row, s_from, j0, jB - 1, false,
                                       las, 0, 0);
                __syncthreads();
                for (int e = tid; e < nbB * nbA; e += NT) {
                    const int m = e / nbA, q = e - m * nbA;
                    las.put(e, M.get((int64_t)(j0 + q) * n + jB + m));
                }
                __syncthreads();
                interchange<A, NB, NT>(M, d, pan, n, jp, nb, cnt, s_row, s_from, jC, n, true, las,
                                       nbA, j0);
                __syncthreads();
            }
        }
        if (bad) break;
        // 5. rows jC.. of the columns right of both panels take both updates
        // (A's multipliers are columns j0.., B's follow), chunk by chunk
        if (nbB == 0) continue;
        const int nq = nbA + nbB;
        for (int r0 = jC; r0 < n; r0 += rch) {
            const int r1 = min(n, r0 + rch), len = r1 - r0;
            for (int e = tid; e < nq * len; e += NT) {
                const int q = e / len, r = e - q * len;
                pan.put(q * rch + r, M.get((int64_t)(j0 + q) * n + r0 + r));
            }
            __syncthreads();
            trailing_update<A, 2 * NB, CB, RB, NT>(M, d, pan, rch, r0, nq, j0, n, jC, n, r0, r1);
            __syncthreads();
        }
    }
    if (bad) {
        if (tid == 0) status[st] = 2;
        return;
    }
    // back substitution, column by column, with d in LDS (the panel's space,
    // free now); the diagonal entry and each thread's first entry of the
    // next column are requested one column ahead
    const LdsVec<A> &sd = pan;
    for (int i = tid; i < n; i += NT) sd.put(i, d.get(i));
    C diag = tid == 0 ? M.get((int64_t)(n - 1) * n + (n - 1)) : A::zero();
    C mc = tid < n - 1 ? M.get((int64_t)(n - 1) * n + tid) : A::zero();
    __syncthreads();
    for (int c = n - 1; c >= 0; --c) {
        if (tid == 0) sd.put(c, A::mul(sd.get(c), A::inv(diag)));
        C diag_n = A::zero(), mc_n = A::zero();
        if (c > 0) {
            if (tid == 0) diag_n = M.get((int64_t)(c - 1) * n + (c - 1));
            if (tid < c - 1) mc_n = M.get((int64_t)(c - 1) * n + tid);
        }
        __syncthreads();
        const C nx = A::neg(sd.get(c));
        if (tid < c) sd.put(tid, A::add(sd.get(tid), A::mul(mc, nx)));
        for (int i = tid + NT; i < c; i += NT)
            sd.put(i, A::add(sd.get(i), A::mul(M.get((int64_t)c * n + i), nx)));
        __syncthreads();
        diag = diag_n;
        mc = mc_n;
    }
    for (int i = tid; i < n; i += NT) d.put(i, sd.get(i));
}

// One step of the pivot search's butterfly among the owners of a column
// (lanes of one aligned group of TPC <= 8 in a wave, all active): keep the
// larger magnitude, the smaller row on ties.  DPP exchanges, no LDS.
template <int OFF>
__device__ __forceinline__ void pivot_step(double &best, int &bi)
{
    const double ob = xor_lane_d<OFF>(best);
    const int oi = xor_lane_i<OFF>(bi);
    if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
    }
}


// Gauss-Jordan elimination with partial pivoting for small complex FP64
// systems (n <= NCOL), one workgroup per start, the matrix in registers:
// thread t owns column c = t / TPC and rows q, q + TPC, q + 2 TPC, ...
// (q = t mod TPC).  Step k:
//   1. the owners of column k find the pivot p (the largest |re| + |im|
//      among the rows not yet pivoted, the smallest row on ties) and write
//      the multipliers l_r = a_rk / a_pk of the other rows to LDS (l_p = 0);
//   2. every thread subtracts l_r a_pc from its entries a_rc of the columns
//      right of k, a_pc coming from the lane of its group that holds row p;
//      the right-hand side (in LDS) likewise.
// Rows are never moved.  After the last step column k holds only its pivot,
// so x_k = b_p / a_pk with no back substitution: about n^3/2 complex
// multiply-adds instead of elimination's n^3/3, all in registers, with one
// barrier per column: the multipliers alternate between two LDS buffers, so
// the owners of column k+1 may look for their pivot while other threads
// still apply step k (no thread reads step k+1's buffer before the barrier
// of step k+1, which every thread reaches only after finishing step k).  A
// failed pivot is recorded as s_piv[k] = -1, read by every thread after that
// step's barrier, so all leave the loop at the same step.
template <int NCOL, int TPC>
__global__ __launch_bounds__(NCOL *TPC) void gj_small_kernel(int64_t n_starts, int32_t n,
                                                             LuPlanes planes, int32_t *status)
{
    constexpr int NT = NCOL * TPC, R = NCOL / TPC;
    static_assert(R <= 32, "the done mask holds 32 rows per thread");
    __shared__ double2 s_l[2][NCOL];  // multipliers of step k in s_l[k & 1]
    __shared__ double2 s_b[NCOL];     // right-hand side
    __shared__ int s_piv[NCOL];       // pivot row of each step, -1: none
    const int64_t st = blockIdx.x;
    if (status[st] != kRunning) return;
    const int tid = threadIdx.x;
    const int c = tid / TPC, q = tid - c * TPC;
    const int lane_base = (tid & 63) - q;  // lane of this column's first owner
    const int64_t mbase = st * (int64_t)n * n + (int64_t)c * n;
    double are[R], aim[R];
    uint32_t done = 0;  // bit i: row q + TPC i already pivoted (or past n)
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int r = q + TPC * i;
        const bool in = c < n && r < n;
        are[i] = in ? planes.J[0][mbase + r] : 0.0;
        aim[i] = in ? planes.J[2][mbase + r] : 0.0;
        if (r >= n) done |= 1u << i;
    }
    for (int r = tid; r < NCOL; r += NT) {
        const int64_t k = st * (int64_t)n + r;
        s_b[r] = r < n ? make_double2(planes.r[0][k], planes.r[2][k]) : make_double2(0.0, 0.0);
    }
    // entry ip of this thread's rows for an index known only at run time
    // (selected, so that the arrays stay in registers)
    auto pick = [&](int ip, double &vr, double &vi) {
        vr = 0.0;
        vi = 0.0;
#pragma unroll
        for (int i = 0; i < R; ++i)
            if (i == ip) {
                vr = are[i];
                vi = aim[i];
            }
    };
    __syncthreads();
    bool bad = false;
    for (int k = 0; k < n; ++k) {
        double2 *const lk = s_l[k & 1];
        if (c == k) {
            double best = -1.0;
            int bi = n;
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const double m = fabs(are[i]) + fabs(aim[i]);
                if (!((done >> i) & 1u) && m > best) {
                    best = m;
                    bi = q + TPC * i;
                }
            }
            // the TPC owners of a column are consecutive lanes of one wave,
            // an aligned group; afterwards all of them hold the same pivot
            static_assert(TPC == 2 || TPC == 4 || TPC == 8, "owners per column");
            pivot_step<1>(best, bi);
            if constexpr (TPC > 2) pivot_step<2>(best, bi);
            if constexpr (TPC > 4) pivot_step<4>(best, bi);
            const bool ok = best > 0.0 && isfinite(best);
            if (q == 0) s_piv[k] = ok ? bi : -1;
            if (ok) {
                // 1 / a_pk, from the lane that holds row p, then the multipliers
                double vr, vi;
                pick(bi / TPC, vr, vi);
                // only this column's owners are active, and all hold bi
                const int src = __builtin_amdgcn_readfirstlane(lane_base + bi % TPC);
                const double pr = read_lane_d(vr, src);
                const double pi = read_lane_d(vi, src);
                const double sc = fmax(fabs(pr), fabs(pi));
                const double sr = pr / sc, si = pi / sc, den = sc * (sr * sr + si * si);
                const double ir = sr / den, ii = -si / den;
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    const int r = q + TPC * i;
                    lk[r] = r == bi ? make_double2(0.0, 0.0)
                                    : make_double2(are[i] * ir - aim[i] * ii, are[i] * ii + aim[i] * ir);
                }
            }
        }
        __syncthreads();
        const int p = s_piv[k];
        if (p < 0) {
            bad = true;
            break;
        }
        const int qp = p % TPC, ip = p / TPC;
        if (c > k && c < n) {
            double vr, vi;
            pick(ip, vr, vi);
            const double pr = __shfl(vr, lane_base + qp, 64), pi = __shfl(vi, lane_base + qp, 64);
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const double2 l = lk[q + TPC * i];
                are[i] = fma(-l.x, pr, fma(l.y, pi, are[i]));
                aim[i] = fma(-l.x, pi, fma(-l.y, pr, aim[i]));
            }
        }
        {
            const double2 bp = s_b[p];
            for (int r = tid; r < n; r += NT) {
                if (r == p) continue;  // zero multiplier; others read s_b[p] now
                const double2 l = lk[r], b = s_b[r];
                s_b[r] = make_double2(fma(-l.x, bp.x, fma(l.y, bp.y, b.x)),
                                      fma(-l.x, bp.y, fma(-l.y, bp.x, b.y)));
            }
        }
        if (q == qp) done |= 1u << ip;
    }
    if (bad) {
        if (tid == 0) status[st] = 2;
        return;
    }
    __syncthreads();  // the last step's right-hand side
    // x_c = b_p / a_pc, p the pivot row of column c, by the owner of row p
    if (c < n) {
        const int p = s_piv[c];
        if (q == p % TPC) {
            double pr, pi;
            pick(p / TPC, pr, pi);
            const double2 b = s_b[p];
            const double sc = fmax(fabs(pr), fabs(pi));
            const double sr = pr / sc, si = pi / sc, den = sc * (sr * sr + si * si);
            const double ir = sr / den, ii = -si / den;
            const int64_t k = st * (int64_t)n + c;
            planes.d[0][k] = b.x * ir - b.y * ii;
            planes.d[2][k] = b.x * ii + b.y * ir;
        }
    }
}

// The same Gauss-Jordan elimination in panels of CPT columns, one wave per
// panel (n <= NCOL, NCOL / CPT waves, one workgroup per start).  Lane q of
// wave w holds rows q, q + 64, ... of columns w CPT .. w CPT + CPT - 1.
//   * Factoring panel P is the work of wave P alone: for each of its
//     columns in turn, the pivot (the largest |re| + |im| over the rows not
//     yet pivoted, the smallest row on ties: a maximum over the wave, then
//     the smallest row that attains it), the multipliers l_r = a_rk / a_pk
//     (l_p = 0) to LDS, and that step applied to the panel's columns right
//     of it, the pivot row's entries taken by readlane.
//   * After one barrier every wave right of the panel applies the panel's
//     steps to its columns in order, and wave 0 to the right-hand side it
//     keeps in registers.  Meanwhile wave P+1, having applied them first,
//     factors panel P+1 into the other multiplier buffer; its wave issues
//     first, since that chain is the serial part of the elimination.
// Every entry sees the same operations in the same order as with one column
// per step (the register kernels above), so the results are the same bit
// for bit; a panel's steps take one barrier instead of one each.  Columns
// past n hold zeros and stay zero; they are updated, never read.
template <int NCOL, int CPT>
__global__ __launch_bounds__((NCOL / CPT) * 64) void gj_panel_kernel(int64_t n_starts, int32_t n,
                                                                      LuPlanes planes,
                                                                      int32_t *status)
{
    constexpr int RPT = NCOL / 64;
    static_assert(NCOL % 64 == 0 && RPT <= 32, "rows per lane, and the done mask");
    __shared__ double2 s_l[2][CPT][NCOL];  // multipliers of a panel's steps; panels alternate
    __shared__ double2 s_b[NCOL];          // right-hand side, for the last step
    __shared__ int s_piv[NCOL];            // pivot row of each column, -1: none
    const int64_t st = blockIdx.x;
    if (status[st] != kRunning) return;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int q = tid & 63;
    const int c0 = w * CPT;
    double are[RPT][CPT], aim[RPT][CPT];
    uint32_t done = 0;  // bit i: row q + 64 i already pivoted (or past n)
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int c = c0 + j;
        const int64_t base = st * (int64_t)n * n + (int64_t)c * n;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int r = q + 64 * i;
            const bool in = c < n && r < n;
            are[i][j] = in ? planes.J[0][base + r] : 0.0;
            aim[i][j] = in ? planes.J[2][base + r] : 0.0;
        }
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i)
        if (q + 64 * i >= n) done |= 1u << i;
    double bre[RPT], bim[RPT];  // wave 0: the right-hand side, rows as above
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int r = q + 64 * i;
        const int64_t k = st * (int64_t)n + r;
        bre[i] = (w == 0 && r < n) ? planes.r[0][k] : 0.0;
        bim[i] = (w == 0 && r < n) ? planes.r[2][k] : 0.0;
    }
    // entry (row slot ip, lane qp) of v, both uniform
    auto at_row = [&](const double (&v)[RPT], int ip, int qp) {
        double x = v[0];
#pragma unroll
        for (int i = 1; i < RPT; ++i)
            if (i == ip) x = v[i];
        return read_lane_d(x, qp);
    };
    // the entries of row (slot ip, lane qp) in this wave's columns jlo ..
    // CPT-1, ip and qp uniform.  One scalar branch per row slot: the empty
    // asm keeps the compiler from merging the two into a vector select of
    // every register before one set of readlanes (32 selects per step).
    static_assert(RPT <= 2, "one or two row slots");
    auto row_entries = [&](int ip, int qp, int jlo, double (&pr)[CPT], double (&pi)[CPT]) {
        if (RPT == 1 || ip == 0) {
#pragma unroll
            for (int c = 0; c < CPT; ++c)
                if (c >= jlo) {
                    pr[c] = read_lane_d(are[0][c], qp);
                    pi[c] = read_lane_d(aim[0][c], qp);
                }
        } else {
            asm volatile("" ::: "memory");
#pragma unroll
            for (int c = 0; c < CPT; ++c)
                if (c >= jlo) {
                    pr[c] = read_lane_d(are[RPT - 1][c], qp);
                    pi[c] = read_lane_d(aim[RPT - 1][c], qp);
                }
        }
    };
    // factor panel P, held by this wave
    auto factor = [&](int P) {
        double2(*lb)[NCOL] = s_l[P & 1];
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int k = P * CPT + j;
            if (k >= n) break;
            double best = -1.0;
            int bi = n;
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const double m = fabs(are[i][j]) + fabs(aim[i][j]);
                if (!((done >> i) & 1u) && m > best) {
                    best = m;
                    bi = q + 64 * i;
                }
            }
            double gm = best;
            gm = max_step<1>(gm);
            gm = max_step<2>(gm);
            gm = max_step<4>(gm);
            gm = max_step<8>(gm);
            gm = max_step<16>(gm);
            gm = max_step<32>(gm);
            int cand = best == gm ? bi : n;
            cand = min_step<1>(cand);
            cand = min_step<2>(cand);
            cand = min_step<4>(cand);
            cand = min_step<8>(cand);
            cand = min_step<16>(cand);
            cand = min_step<32>(cand);
            const int p = __builtin_amdgcn_readfirstlane(cand);
            const bool ok = __builtin_amdgcn_readfirstlane((int)(gm > 0.0 && isfinite(gm))) != 0;
            if (q == 0) s_piv[k] = ok ? p : -1;
            if (!ok) break;
            const int qp = p & 63, ip = p >> 6;
            // row p in columns j .. CPT-1: the pivot, then the entries the
            // step subtracts from this panel's columns right of it
            double rowr[CPT], rowi[CPT];
            row_entries(ip, qp, j, rowr, rowi);
            const double pr = rowr[j], pi = rowi[j];
            const double sc = fmax(fabs(pr), fabs(pi));
            const double sr = pr / sc, si = pi / sc, den = sc * (sr * sr + si * si);
            const double ir = sr / den, ii = -si / den;
            double lr[RPT], li[RPT];
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int r = q + 64 * i;
                const double cr = are[i][j], ci = aim[i][j];
                const double mr = cr * ir - ci * ii, mi = cr * ii + ci * ir;
                const bool z = r == p;
                lr[i] = z ? 0.0 : mr;
                li[i] = z ? 0.0 : mi;
                lb[j][r] = make_double2(lr[i], li[i]);
            }
#pragma unroll
            for (int jj = j + 1; jj < CPT; ++jj) {
                const double prr = rowr[jj], pri = rowi[jj];
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    are[i][jj] = fma(-lr[i], prr, fma(li[i], pri, are[i][jj]));
                    aim[i][jj] = fma(-lr[i], pri, fma(-li[i], prr, aim[i][jj]));
                }
            }
            if (q == qp) done |= 1u << ip;
        }
    };
    const int NP = (n + CPT - 1) / CPT;
    if (w == 0) factor(0);
    bool bad = false;
    for (int P = 0; P < NP; ++P) {
        __syncthreads();
        if (w == P + 1)
            __builtin_amdgcn_s_setprio(3);
        else
            __builtin_amdgcn_s_setprio(0);
        const int kend = min(n - P * CPT, CPT);
        int piv[CPT];
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            piv[j] = j < kend ? __builtin_amdgcn_readfirstlane(s_piv[P * CPT + j]) : 0;
            if (piv[j] < 0) bad = true;
        }
        if (bad) break;
        double2(*lb)[NCOL] = s_l[P & 1];
        if (w > P) {
            double2 ln[RPT];
#pragma unroll
            for (int i = 0; i < RPT; ++i) ln[i] = lb[0][q + 64 * i];
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                if (j >= kend) break;
                const int p = piv[j], qp = p & 63, ip = p >> 6;
                double2 l[RPT];
#pragma unroll
                for (int i = 0; i < RPT; ++i) l[i] = ln[i];
                if (j + 1 < CPT)
#pragma unroll
                    for (int i = 0; i < RPT; ++i) ln[i] = lb[j + 1][q + 64 * i];
                double prr[CPT], pri[CPT];
                row_entries(ip, qp, 0, prr, pri);
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
#pragma unroll
                    for (int i = 0; i < RPT; ++i) {
                        are[i][c] = fma(-l[i].x, prr[c], fma(l[i].y, pri[c], are[i][c]));
                        aim[i][c] = fma(-l[i].x, pri[c], fma(-l[i].y, prr[c], aim[i][c]));
                    }
                }
                if (q == qp) done |= 1u << ip;
            }
        }
        if (w == 0) {
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                if (j >= kend) break;
                const int p = piv[j], qp = p & 63, ip = p >> 6;
                const double bpr = at_row(bre, ip, qp), bpi = at_row(bim, ip, qp);
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const int r = q + 64 * i;
                    if (r == p) continue;  // zero multiplier
                    const double2 l = lb[j][r];
                    bre[i] = fma(-l.x, bpr, fma(l.y, bpi, bre[i]));
                    bim[i] = fma(-l.x, bpi, fma(-l.y, bpr, bim[i]));
                }
            }
        }
        if (w == P + 1 && P + 1 < NP) factor(P + 1);
    }
    __builtin_amdgcn_s_setprio(0);
    if (bad) {
        if (tid == 0) status[st] = 2;
        return;
    }
    if (w == 0) {
#pragma unroll
        for (int i = 0; i < RPT; ++i) s_b[q + 64 * i] = make_double2(bre[i], bim[i]);
    }
    __syncthreads();
    // x_c = b_p / a_pc, p the pivot row of column c, by the lane that holds row p
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int c = c0 + j;
        if (c >= n) continue;
        const int p = s_piv[c];
        if (q != (p & 63)) continue;
        const int ipc = p >> 6;
        double pr = are[0][j], pi = aim[0][j];
#pragma unroll
        for (int i = 1; i < RPT; ++i)
            if (i == ipc) {
                pr = are[i][j];
                pi = aim[i][j];
            }
        const double2 b = s_b[p];
        const double sc = fmax(fabs(pr), fabs(pi));
        const double sr = pr / sc, si = pi / sc, den = sc * (sr * sr + si * si);
        const double ir = sr / den, ii = -si / den;
        const int64_t kk = st * (int64_t)n + c;
        planes.d[0][kk] = b.x * ir - b.y * ii;
        planes.d[2][kk] = b.x * ii + b.y * ir;
    }
}

// Panel width: 16 columns in FP64 and 8 in double-double, or fewer when
// the panel (width x n complex values) and the kernel's static arrays would
// not fit in LDS; 0 if none fits.
static int lu_panel(int prec, int32_t n)
{
    static_assert(kLdsBytes == (size_t)kMaxLds, "one LDS size");
    return prec == 0 ? lu_panel_width(sizeof(Arith64::C), n, 16)
                     : lu_panel_width(sizeof(ArithDD::C), n, 8);
}

// Threads per workgroup: 512 for n >= 256 (two waves per SIMD keep the
// long trailing updates busy; the registers of both arithmetics allow it
// with panels of at most 16 FP64 or 8 double-double columns), else 256.
static int lu_threads(int32_t n) { return n >= 256 ? 512 : 256; }

template <class A, int NT>
static const void *lu_kernel_nt(int nb)
{
    // double-double panels are at most 8 wide (lu_panel)
    switch (nb) {
    case 16:
        if constexpr (std::is_same<A, Arith64>::value)
            return reinterpret_cast<const void *>(lu_solve_kernel<A, 16, NT>);
        else
            return nullptr;
    case 8: return reinterpret_cast<const void *>(lu_solve_kernel<A, 8, NT>);
    case 4: return reinterpret_cast<const void *>(lu_solve_kernel<A, 4, NT>);
    default: return reinterpret_cast<const void *>(lu_solve_kernel<A, 2, NT>);
    }
}

static const void *lu_kernel(int prec, int nb, int threads)
{
    if (prec != 0)
        return threads == 512 ? lu_kernel_nt<ArithDD, 512>(nb) : lu_kernel_nt<ArithDD, 256>(nb);
    return threads == 512 ? lu_kernel_nt<Arith64, 512>(nb) : lu_kernel_nt<Arith64, 256>(nb);
}

hipError_t launch_lu_solve(int prec, int64_t n_starts, int32_t n, double *const J[4],
                           const double *const r[4], double *const d[4], int32_t *status,
                           hipStream_t stream)
{
    if (n_starts <= 0) return hipSuccess;
    if (prec == 0 && n <= 128) {
        LuPlanes pl;
        for (int q = 0; q < 4; ++q) {
            pl.J[q] = J[q];
            pl.r[q] = r[q];
            pl.d[q] = d[q];
        }
        if (n <= 32)
            hipLaunchKernelGGL((gj_small_kernel<32, 4>), dim3((unsigned)n_starts), dim3(128), 0,
                               stream, n_starts, n, pl, status);
        else if (n <= 64)
            hipLaunchKernelGGL((gj_panel_kernel<64, 8>), dim3((unsigned)n_starts), dim3(512), 0,
                               stream, n_starts, n, pl, status);
        else
            hipLaunchKernelGGL((gj_panel_kernel<128, 8>), dim3((unsigned)n_starts), dim3(1024),
                               0, stream, n_starts, n, pl, status);
        return hipGetLastError();
    }
    const int nb = lu_panel(prec, n);
    if (nb == 0) return hipErrorInvalidValue;
    LuPlanes pl;
    for (int q = 0; q < 4; ++q) {
        pl.J[q] = J[q];
        pl.r[q] = r[q];
        pl.d[q] = d[q];
    }
    const size_t lds = (prec == 0 ? sizeof(Arith64::C) : sizeof(ArithDD::C)) * (size_t)nb * n;
    void *args[] = {&n_starts, &n, &pl, &status};
    const int threads = lu_threads(n);
    return hipLaunchKernel(lu_kernel(prec, nb, threads), dim3((unsigned)n_starts),
                           dim3((unsigned)threads), args, lds, stream);
}

bool lu_solve_fits(int prec, int32_t n) { return lu_panel(prec, n) > 0; }

// ---------------------------------------------------------------------------
// update and initialization
// ---------------------------------------------------------------------------

template <int PREC>
__global__ void update_kernel(int64_t n_starts, int32_t n, UpdPlanes pl, const int32_t *status,
                              int32_t *iters)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_starts * n) return;
    const int64_t s = k / n;
    if (status[s] != kRunning) return;
    if constexpr (PREC == 2) {
        // quad-double x, FP64 step
        using IO = Io<ArithQD>;
        const ArithQD::C x = IO::load(pl.x, k);
        const ArithQD::C step{{pl.d[0][k], 0.0, 0.0, 0.0}, {pl.d[2][k], 0.0, 0.0, 0.0}};
        IO::store(pl.x, k, ArithQD::add(x, ArithQD::neg(step)));
        if (k % n == 0) iters[s] += 1;
        return;
    }
    dd re{pl.x[0][k], pl.x[1][k]}, im{pl.x[2][k], pl.x[3][k]};
    dd dre, dim;
    if (PREC == 0) {
        dre = {pl.d[0][k], 0.0};
        dim = {pl.d[2][k], 0.0};
    } else {
        dre = {pl.d[0][k], pl.d[1][k]};
        dim = {pl.d[2][k], pl.d[3][k]};
    }
    re = dw_add(re, dw_neg(dre));
    im = dw_add(im, dw_neg(dim));
    pl.x[0][k] = re.hi;
    pl.x[1][k] = re.lo;
    pl.x[2][k] = im.hi;
    pl.x[3][k] = im.lo;
    if (k % n == 0) iters[s] += 1;
}

hipError_t launch_update(int prec, int64_t n_starts, int32_t n, double *const *x,
                         const double *const d[4], const int32_t *status, int32_t *iters,
                         hipStream_t stream)
{
    const int64_t total = n_starts * (int64_t)n;
    if (total <= 0) return hipSuccess;
    UpdPlanes pl{};
    for (int q = 0; q < (prec == 2 ? 8 : 4); ++q) pl.x[q] = x[q];
    for (int q = 0; q < 4; ++q) pl.d[q] = d[q];
    const unsigned blocks = (unsigned)((total + 255) / 256);
    if (prec == 0)
        hipLaunchKernelGGL(update_kernel<0>, dim3(blocks), dim3(256), 0, stream, n_starts, n, pl,
                           status, iters);
    else if (prec == 1)
        hipLaunchKernelGGL(update_kernel<1>, dim3(blocks), dim3(256), 0, stream, n_starts, n, pl,
                           status, iters);
    else
        hipLaunchKernelGGL(update_kernel<2>, dim3(blocks), dim3(256), 0, stream, n_starts, n, pl,
                           status, iters);
    return hipGetLastError();
}

__global__ void newton_init_kernel(int64_t n_starts, int32_t *status, int32_t *iters)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_starts) return;
    status[s] = kRunning;
    iters[s] = 0;
}

hipError_t launch_newton_init(int64_t n_starts, int32_t *status, int32_t *iters, hipStream_t stream)
{
    if (n_starts <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n_starts + 255) / 256);
    hipLaunchKernelGGL(newton_init_kernel, dim3(blocks), dim3(256), 0, stream, n_starts, status,
                       iters);
    return hipGetLastError();
}

hipError_t newton_kernels_init()
{
    // best effort: a refusal shows up later as a launch error
    std::vector<const void *> ks{
        reinterpret_cast<const void *>(resid_kernel<ArithDD, kResidThreads>),
        reinterpret_cast<const void *>(resid_kernel<ArithQD, kResidThreadsQD>)};
    for (int nb : {16, 8, 4, 2})
        for (int prec : {0, 1})
            for (int threads : {256, 512})
                if (const void *k = lu_kernel(prec, nb, threads)) ks.push_back(k);
    for (const void *k : ks)
        if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds) !=
            hipSuccess)
            (void)hipGetLastError();
    return hipSuccess;
}

}  // namespace pe
