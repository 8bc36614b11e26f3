// Device helpers shared by the kernels: lane exchanges inside a wave,
// lane-group products, and loads/stores of complex values in plane layout.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "dd.hpp"
#include "qd.hpp"

namespace pe {

// Exchange with lane (lane ^ m) of the same wave.  Masks 1, 2 and 8 are one
// DPP move inside rows of 16 lanes (quad_perm [1,0,3,2], quad_perm
// [2,3,0,1], row_ror:8); mask 4 is two DPP moves into one register, banks 0
// and 2 of each row (lane bit 2 clear) from row_shl:4, banks 1 and 3 from
// row_shr:4, each under a bank mask, so every lane reads a lane of its own
// row and no select is needed; masks 16 and 32 use gfx950's row swaps
// (v_permlane16_swap / v_permlane32_swap with both operands the value: the
// first result holds, in the odd rows, the even rows' values, the second
// the reverse).  All lanes of the wave must be active.
template <int M>
__device__ __forceinline__ int xor_lane_i(int v)
{
    if constexpr (M == 1) {
        return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
    } else if constexpr (M == 2) {
        return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
    } else if constexpr (M == 4) {
        const int up = __builtin_amdgcn_mov_dpp(v, 0x104, 0xF, 0x5, false);  // from lane+4
        return __builtin_amdgcn_update_dpp(up, v, 0x114, 0xF, 0xA, false);   // from lane-4
    } else if constexpr (M == 8) {
        return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);
    } else if constexpr (M == 16) {
        const auto s = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (int)((threadIdx.x & 16) ? s[0] : s[1]);
    } else {
        static_assert(M == 32, "lane masks are powers of two below 64");
        const auto s = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (int)((threadIdx.x & 32) ? s[0] : s[1]);
    }
}

template <int M>
__device__ __forceinline__ double xor_lane_d(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = xor_lane_i<M>((int)(b & 0xFFFFFFFFll));
    const int hi = xor_lane_i<M>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int M>
__device__ __forceinline__ ArithDD::C xor_lane_c(const ArithDD::C &v)
{
    return {{xor_lane_d<M>(v.re.hi), xor_lane_d<M>(v.re.lo)},
            {xor_lane_d<M>(v.im.hi), xor_lane_d<M>(v.im.lo)}};
}

template <int M>
__device__ __forceinline__ Arith64::C xor_lane_c(const Arith64::C &v)
{
    return {xor_lane_d<M>(v.re), xor_lane_d<M>(v.im)};
}

template <int M>
__device__ __forceinline__ qd xor_lane_q(const qd &v)
{
    return {xor_lane_d<M>(v.x0), xor_lane_d<M>(v.x1), xor_lane_d<M>(v.x2), xor_lane_d<M>(v.x3)};
}

template <int M>
__device__ __forceinline__ ArithQD::C xor_lane_c(const ArithQD::C &v)
{
    return {xor_lane_q<M>(v.re), xor_lane_q<M>(v.im)};
}

// Both results of a row swap of every dword of a value (M = 16 or 32): lane
// by lane, one holds its own value and the other the value of lane ^ M.
template <int M>
__device__ __forceinline__ void swap_rows_d(double v, double &a, double &b)
{
    const long long x = __double_as_longlong(v);
    const int lo = (int)(x & 0xFFFFFFFFll), hi = (int)(x >> 32);
    const auto sl = M == 16 ? __builtin_amdgcn_permlane16_swap(lo, lo, false, false)
                            : __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto sh = M == 16 ? __builtin_amdgcn_permlane16_swap(hi, hi, false, false)
                            : __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    a = __longlong_as_double(((long long)(int)sh[0] << 32) | (unsigned int)sl[0]);
    b = __longlong_as_double(((long long)(int)sh[1] << 32) | (unsigned int)sl[1]);
}

template <int M>
__device__ __forceinline__ void swap_rows_c(const ArithDD::C &v, ArithDD::C &a, ArithDD::C &b)
{
    swap_rows_d<M>(v.re.hi, a.re.hi, b.re.hi);
    swap_rows_d<M>(v.re.lo, a.re.lo, b.re.lo);
    swap_rows_d<M>(v.im.hi, a.im.hi, b.im.hi);
    swap_rows_d<M>(v.im.lo, a.im.lo, b.im.lo);
}

template <int M>
__device__ __forceinline__ void swap_rows_c(const Arith64::C &v, Arith64::C &a, Arith64::C &b)
{
    swap_rows_d<M>(v.re, a.re, b.re);
    swap_rows_d<M>(v.im, a.im, b.im);
}

// v + (v of lane lane ^ M), for arithmetic whose sum gives the same bits in
// either operand order (FP64 addition; the double-word sum: TwoSum's error
// is the exact rounding error whatever the order, and the low words are
// added commutatively).  Across rows the two swap results are added
// directly, with no select of the partner's half; results equal
// A::sum(v, xor_lane_c<M>(v)) bit for bit.
template <class A, int M>
__device__ __forceinline__ typename A::C sum_xor(const typename A::C &v)
{
    if constexpr ((M == 16 || M == 32) && (std::is_same<A, ArithDD>::value ||
                                           std::is_same<A, Arith64>::value)) {
        typename A::C a, b;
        swap_rows_c<M>(v, a, b);
        return A::sum(a, b);
    } else {
        return A::sum(v, xor_lane_c<M>(v));
    }
}

// runtime mask (uniform across the wave)
template <class A>
__device__ __forceinline__ typename A::C sum_xor_c(const typename A::C &v, int m)
{
    switch (m) {
    case 1: return sum_xor<A, 1>(v);
    case 2: return sum_xor<A, 2>(v);
    case 4: return sum_xor<A, 4>(v);
    case 8: return sum_xor<A, 8>(v);
    case 16: return sum_xor<A, 16>(v);
    default: return sum_xor<A, 32>(v);
    }
}

// runtime mask (uniform across the wave)
template <class C>
__device__ __forceinline__ C shfl_xor_c(const C &v, int m)
{
    switch (m) {
    case 1: return xor_lane_c<1>(v);
    case 2: return xor_lane_c<2>(v);
    case 4: return xor_lane_c<4>(v);
    case 8: return xor_lane_c<8>(v);
    case 16: return xor_lane_c<16>(v);
    default: return xor_lane_c<32>(v);
    }
}

// Butterfly over a group of L consecutive lanes (L a power of two): each
// lane receives the exclusive product E of the other lanes' values cf * P.
struct LaneGroup {
    int L;
    // E = product over the other lanes of the group of cf * P
    template <class A>
    __device__ __forceinline__ void combine(const typename A::C &cf, const typename A::C &P,
                                            typename A::C &E, bool &have_E) const
    {
        using C = typename A::C;
        have_E = L > 1;
        if (!have_E) return;
        C blk = A::mul(cf, P);
        for (int d = 1; d < L; d <<= 1) {
            const C other = shfl_xor_c(blk, d);
            E = (d == 1) ? other : A::mul(E, other);
            if (2 * d < L) blk = A::mul(blk, other);
        }
    }
};

// An array of complex values in LDS, in 16-byte pieces read and written
// with one 128-bit access each.  A complex double-double value is split
// over two planes, (re.hi, re.lo) and (im.hi, im.lo): lanes at consecutive
// entries then cover all 64 banks in one access, and random entries
// collide half as often as with 32-byte entries.
template <class A>
struct LdsVec;

template <>
struct LdsVec<ArithDD> {
    double2 *re, *im;  // the planes, count entries each
    __device__ __forceinline__ ArithDD::C get(int i) const
    {
        const double2 r = re[i], m = im[i];
        return {{r.x, r.y}, {m.x, m.y}};
    }
    __device__ __forceinline__ void put(int i, const ArithDD::C &v) const
    {
        re[i] = make_double2(v.re.hi, v.re.lo);
        im[i] = make_double2(v.im.hi, v.im.lo);
    }
    // the array of `count` entries at raw, and the LDS that follows it
    __device__ __forceinline__ static LdsVec at(double2 *raw, int count, double2 *&next)
    {
        next = raw + 2 * (size_t)count;
        return {raw, raw + count};
    }
};

template <>
struct LdsVec<ArithQD> {
    double2 *p;  // four planes of count entries: re (x0, x1), re (x2, x3), im (x0, x1), im (x2, x3)
    int count;
    __device__ __forceinline__ ArithQD::C get(int i) const
    {
        const double2 a = p[i], b = p[count + i], c = p[2 * count + i], d = p[3 * count + i];
        return {{a.x, a.y, b.x, b.y}, {c.x, c.y, d.x, d.y}};
    }
    __device__ __forceinline__ void put(int i, const ArithQD::C &v) const
    {
        p[i] = make_double2(v.re.x0, v.re.x1);
        p[count + i] = make_double2(v.re.x2, v.re.x3);
        p[2 * count + i] = make_double2(v.im.x0, v.im.x1);
        p[3 * count + i] = make_double2(v.im.x2, v.im.x3);
    }
    __device__ __forceinline__ static LdsVec at(double2 *raw, int count, double2 *&next)
    {
        next = raw + 4 * (size_t)count;
        return {raw, count};
    }
};

template <>
struct LdsVec<Arith64> {
    double2 *v;
    __device__ __forceinline__ Arith64::C get(int i) const
    {
        const double2 r = v[i];
        return {r.x, r.y};
    }
    __device__ __forceinline__ void put(int i, const Arith64::C &c) const { v[i] = make_double2(c.re, c.im); }
    __device__ __forceinline__ static LdsVec at(double2 *raw, int count, double2 *&next)
    {
        next = raw + count;
        return {raw};
    }
};

template <class A>
struct Io;

template <>
struct Io<ArithDD> {
    using C = ArithDD::C;
    __device__ __forceinline__ static C load(const double *const *pl, int64_t i)
    {
        return {{pl[0][i], pl[1][i]}, {pl[2][i], pl[3][i]}};
    }
    __device__ __forceinline__ static void store(double *const *pl, int64_t i, const C &v)
    {
        pl[0][i] = v.re.hi;
        pl[1][i] = v.re.lo;
        pl[2][i] = v.im.hi;
        pl[3][i] = v.im.lo;
    }
    __device__ __forceinline__ static C coef(const double *c, int64_t s)
    {
        const double *p = c + 4 * s;
        return {{p[0], p[1]}, {p[2], p[3]}};
    }
    __device__ __forceinline__ static void put(double *g, const C &v)
    {
        g[0] = v.re.hi;
        g[1] = v.re.lo;
        g[2] = v.im.hi;
        g[3] = v.im.lo;
    }
    __device__ __forceinline__ static C get(const double *g) { return {{g[0], g[1]}, {g[2], g[3]}}; }
};

// quad-double values in eight planes: re x0..x3, then im x0..x3; the
// system's coefficients are double-double (their low words are zero here)
template <>
struct Io<ArithQD> {
    using C = ArithQD::C;
    __device__ __forceinline__ static C load(const double *const *pl, int64_t i)
    {
        return {{pl[0][i], pl[1][i], pl[2][i], pl[3][i]}, {pl[4][i], pl[5][i], pl[6][i], pl[7][i]}};
    }
    __device__ __forceinline__ static void store(double *const *pl, int64_t i, const C &v)
    {
        pl[0][i] = v.re.x0;
        pl[1][i] = v.re.x1;
        pl[2][i] = v.re.x2;
        pl[3][i] = v.re.x3;
        pl[4][i] = v.im.x0;
        pl[5][i] = v.im.x1;
        pl[6][i] = v.im.x2;
        pl[7][i] = v.im.x3;
    }
    __device__ __forceinline__ static C coef(const double *c, int64_t s)
    {
        const double *p = c + 4 * s;
        return {{p[0], p[1], 0.0, 0.0}, {p[2], p[3], 0.0, 0.0}};
    }
    __device__ __forceinline__ static void put(double *g, const C &v)
    {
        g[0] = v.re.x0;
        g[1] = v.re.x1;
        g[2] = v.re.x2;
        g[3] = v.re.x3;
        g[4] = v.im.x0;
        g[5] = v.im.x1;
        g[6] = v.im.x2;
        g[7] = v.im.x3;
    }
    __device__ __forceinline__ static C get(const double *g)
    {
        return {{g[0], g[1], g[2], g[3]}, {g[4], g[5], g[6], g[7]}};
    }
};

template <>
struct Io<Arith64> {
    using C = Arith64::C;
    __device__ __forceinline__ static C load(const double *const *pl, int64_t i)
    {
        return {pl[0][i], pl[2][i]};
    }
    __device__ __forceinline__ static void store(double *const *pl, int64_t i, const C &v)
    {
        pl[0][i] = v.re;
        pl[2][i] = v.im;
    }
    __device__ __forceinline__ static C coef(const double *c, int64_t s)
    {
        const double *p = c + 4 * s;
        return {p[0], p[2]};
    }
    __device__ __forceinline__ static void put(double *g, const C &v)
    {
        g[0] = v.re;
        g[1] = v.im;
    }
    __device__ __forceinline__ static C get(const double *g) { return {g[0], g[1]}; }
};

}  // namespace pe
