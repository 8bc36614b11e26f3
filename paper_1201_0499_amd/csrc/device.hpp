// Device helpers shared by the kernels: lane exchanges inside a wave,
// lane-group products, and loads/stores of complex values in plane layout.
#pragma once

#include <hip/hip_runtime.h>

#include "dd.hpp"
#include "qd.hpp"

namespace pe {

// Exchange with lane (lane ^ m) of the same wave.  Masks 1, 2, 4 and 8 use
// DPP lane permutations inside rows of 16 lanes (quad_perm [1,0,3,2] and
// [2,3,0,1]; row_ror by 4/12 selected by lane bit 2; row_ror by 8); masks 16
// and 32 use gfx950's row swaps (v_permlane16_swap / v_permlane32_swap with
// both operands the value: the first result holds, in the odd rows, the even
// rows' values, the second the reverse).  All lanes of the wave must be
// active.
template <int M>
__device__ __forceinline__ int xor_lane_i(int v)
{
    if constexpr (M == 1) {
        return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);
    } else if constexpr (M == 2) {
        return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);
    } else if constexpr (M == 4) {
        const int down = __builtin_amdgcn_update_dpp(0, v, 0x124, 0xF, 0xF, false);  // from lane-4
        const int up = __builtin_amdgcn_update_dpp(0, v, 0x12C, 0xF, 0xF, false);    // from lane+4
        return (threadIdx.x & 4) ? down : up;
    } else if constexpr (M == 8) {
        return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false);
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
