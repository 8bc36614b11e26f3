// The paper's own three-kernel organisation of the evaluation (Section 3),
// kept for comparison with the fused kernel of eval.hip on the same GPU:
//
//   1. common factors: one thread per (point, monomial) raises each of its
//      variables to a - 1 by repeated multiplication, with no shared power
//      table, and writes CF to global memory (Section 3.1);
//   2. monomial terms: one thread per (point, monomial) forms the
//      Speelpenning partials with forward and backward products, multiplies
//      them by CF and by k + 1 coefficients prescaled on the host (c a_j for
//      the partials, c for the value; Section 3.2), and scatters them into a
//      dense term array holding n + 1 rows of m entries per polynomial, zero
//      where a variable does not occur (Section 3.3);
//   3. summation: one thread per output adds its m entries in monomial
//      order (Section 3.3).
//
// The dense array is zeroed once when it is allocated; the entries the
// terms kernel writes are the same at every evaluation, so the zeros stay.
#include <hip/hip_runtime.h>

#include "ablation.hpp"
#include "device.hpp"
#include "packing.hpp"

namespace pe {

namespace {

template <class A>
struct PlaneIo;

template <>
struct PlaneIo<ArithDD> {
    using C = ArithDD::C;
    __device__ static C get(const double *p, int64_t i, int64_t stride)
    {
        return {{p[i], p[i + stride]}, {p[i + 2 * stride], p[i + 3 * stride]}};
    }
    __device__ static void put(double *p, int64_t i, int64_t stride, const C &v)
    {
        p[i] = v.re.hi;
        p[i + stride] = v.re.lo;
        p[i + 2 * stride] = v.im.hi;
        p[i + 3 * stride] = v.im.lo;
    }
};

template <>
struct PlaneIo<Arith64> {
    using C = Arith64::C;
    __device__ static C get(const double *p, int64_t i, int64_t stride) { return {p[i], p[i + stride]}; }
    __device__ static void put(double *p, int64_t i, int64_t stride, const C &v)
    {
        p[i] = v.re;
        p[i + stride] = v.im;
    }
};

template <class A>
__global__ __launch_bounds__(256) void cf_kernel(const AblationArgs a)
{
    using C = typename A::C;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.n_points * a.n_monos) return;
    const int64_t pt = e / a.n_monos, s = e - pt * a.n_monos;
    C cf = A::one();
    for (int j = a.mono_start[s]; j < a.mono_start[s + 1]; ++j) {
        const uint32_t w = a.word[j];
        const C x = Io<A>::load(a.x, pt * a.n_vars + (int)(w & kPosMask));
        for (int r = (int)(w >> kExpShift); r > 0; --r) cf = A::mul(cf, x);
    }
    PlaneIo<A>::put(a.cf, e, a.n_points * a.n_monos, cf);
}

template <class A, int KMAX>
__global__ __launch_bounds__(256) void terms_kernel(const AblationArgs a)
{
    using C = typename A::C;
    constexpr int W = A::kWords;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.n_points * a.n_monos) return;
    const int64_t pt = e / a.n_monos, s = e - pt * a.n_monos;
    const int j0 = a.mono_start[s], k = a.mono_start[s + 1] - j0;
    const int p = a.mono_poly[s];
    const int64_t s0 = a.poly_start[p], m = a.poly_start[p + 1] - s0;
    const int np1 = a.n_vars + 1;
    // this point's block of the dense array, polynomial p: rows o = 0..n, m entries each
    C *const blk = reinterpret_cast<C *>(a.mons) + pt * (int64_t)np1 * a.n_monos + s0 * np1;
    const int64_t col = s - s0;
    const C cf = PlaneIo<A>::get(a.cf, e, a.n_points * a.n_monos);
    // prescaled coefficients of this monomial: c a_t for t < k, then c
    // (four words each; FP64 reads the leading ones)
    const double *pc = a.pcoef + (int64_t)a.pcoef_start[s] * 4;
    auto coef = [&](int t) -> C {
        const double *q = pc + (int64_t)t * 4;
        if constexpr (W == 4)
            return C{{q[0], q[1]}, {q[2], q[3]}};
        else
            return C{q[0], q[2]};
    };
    C x[KMAX], fw[KMAX];
    int pos[KMAX];
#pragma unroll
    for (int t = 0; t < KMAX; ++t)
        if (t < k) {
            const uint32_t w = a.word[j0 + t];
            pos[t] = (int)(w & kPosMask);
            x[t] = Io<A>::load(a.x, pt * a.n_vars + pos[t]);
        }
    if (k == 0) {
        blk[(int64_t)a.n_vars * m + col] = coef(0);
        return;
    }
    // forward products fw[t] = x_0 ... x_{t-1}, then the backward product
    // runs from the last variable down
    C prod = A::one();
#pragma unroll
    for (int t = 0; t < KMAX; ++t)
        if (t < k) {
            fw[t] = prod;
            prod = A::mul(prod, x[t]);
        }
    blk[(int64_t)a.n_vars * m + col] = A::mul(A::mul(prod, cf), coef(k));
    C bw = A::one();
#pragma unroll
    for (int t = KMAX - 1; t >= 0; --t)
        if (t < k) {
            const C st = A::mul(fw[t], bw);  // product of the other variables
            blk[(int64_t)pos[t] * m + col] = A::mul(A::mul(st, cf), coef(t));
            bw = A::mul(bw, x[t]);
        }
}

template <class A>
__global__ __launch_bounds__(256) void sum_kernel(const AblationArgs a)
{
    using C = typename A::C;
    const int np1 = a.n_vars + 1;
    const int64_t outs = (int64_t)a.n_polys * np1;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.n_points * outs) return;
    const int64_t pt = e / outs;
    const int64_t r = e - pt * outs;
    const int p = (int)(r / np1), o = (int)(r - (int64_t)p * np1);
    const int64_t s0 = a.poly_start[p], m = a.poly_start[p + 1] - s0;
    const C *row = reinterpret_cast<const C *>(a.mons) + pt * (int64_t)np1 * a.n_monos + s0 * np1 +
                   (int64_t)o * m;
    C v = A::zero();
    for (int64_t i = 0; i < m; ++i) v = A::add(v, row[i]);
    if (o == a.n_vars)
        Io<A>::store(a.f, pt * a.n_polys + p, v);
    else if (a.J[0])
        Io<A>::store(a.J, pt * (int64_t)a.n_vars * a.n_polys + (int64_t)o * a.n_polys + p, v);
}

unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <class A>
hipError_t launch_all(const AblationArgs &a, int kmax, hipStream_t stream)
{
    const int64_t units = a.n_points * a.n_monos;
    if (units > 0) {
        hipLaunchKernelGGL(cf_kernel<A>, dim3(blocks_for(units, 256)), dim3(256), 0, stream, a);
        if (kmax <= 8)
            hipLaunchKernelGGL((terms_kernel<A, 8>), dim3(blocks_for(units, 256)), dim3(256), 0,
                               stream, a);
        else if (kmax <= 16)
            hipLaunchKernelGGL((terms_kernel<A, 16>), dim3(blocks_for(units, 256)), dim3(256), 0,
                               stream, a);
        else
            hipLaunchKernelGGL((terms_kernel<A, 32>), dim3(blocks_for(units, 256)), dim3(256), 0,
                               stream, a);
    }
    const int64_t outs = a.n_points * (int64_t)a.n_polys * (a.n_vars + 1);
    if (outs > 0)
        hipLaunchKernelGGL(sum_kernel<A>, dim3(blocks_for(outs, 256)), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ablation(int prec, const AblationArgs &a, int kmax, hipStream_t stream)
{
    return prec == 1 ? launch_all<ArithDD>(a, kmax, stream) : launch_all<Arith64>(a, kmax, stream);
}

}  // namespace pe
