// Complex double-double and complex FP64 arithmetic for the evaluation
// kernels, usable on the host (for tests and operation counting) and on
// gfx950.
//
// Double-double ("double-word") numbers x = hi + lo with |lo| <= ulp(hi)/2,
// the extended precision the paper adopts for path tracking (Section 1,
// double double arithmetic; Section 3.2 sizes the kernels for it).  The
// building blocks are error-free transformations on FP64:
//   two_sum       Knuth / Moller: s + e == a + b exactly,
//   fast_two_sum  Dekker: the same when |a| >= |b|,
//   two_prod      p + e == a * b exactly, with one fused multiply-add,
// and the double-word algorithms of Joldes, Muller & Popescu (ACM TOMS
// 44(2), 2017): the accurate sum (relative error <= 3u^2) and the product
// with FMA (relative error <= 5u^2), u = 2^-53.
//
// The complex product used by the kernels (ArithDD::mul) is fused: each of
// the real and imaginary parts is a two-term dot product ah*bh +- ch*dh
// formed exactly with two FMA TwoProducts and one TwoSum, plus the
// first-order cross terms accumulated in one FP64 chain of FMAs, and
// renormalized with a final FastTwoSum.  It costs 38 FP64 instructions
// instead of 76 for four double-word products and two double-word sums.
// Error of one part, with M = |a_re||b_re| + |a_im||b_im|: the two leading
// products and their sum are exact; the six first-order terms (two
// TwoProduct errors, the TwoSum error and four hi*lo products) are each at
// most u*M in size, so the FP64 chain adding them, t, rounds six times on
// partial sums below 4uM, i.e. at most 24 u^2 M; the dropped lo*lo products
// add at most u^2 M.  The final FastTwoSum(s, t) is exact when |s| >= |t|;
// otherwise the two leading products cancelled to within 4uM, so
// |s + t| < 8uM and the renormalization errs by at most u|s + t|, below
// 8 u^2 M, which the bound's slack covers: total below 25 u^2 M (the tests
// check it against exact rationals, cancellation included).
//
// Sums of many terms (the segmented summation, the value and residual
// reductions) use the sloppy double-word sum: one TwoSum of the high words,
// the low words added in FP64, one FastTwoSum; 11 instructions instead of
// 20.  Its error is bounded in absolute terms, by 4 u^2 (|x| + |y|), not
// relative to |x + y|; over a sum of N terms that is the same order as the
// accurate sum's (both are bounded by a multiple of u^2 times the sum of
// magnitudes), which is the measure the evaluation is judged by.  The
// elimination in the Newton solver keeps the accurate sum.  Runs of terms
// (pieces of the segmented summation, a lane's monomials in the residual)
// use the cascaded accumulator DWAcc below.
//
// All code using these must be compiled with -ffp-contract=off: a fused
// multiply-add introduced by the compiler into two_sum or fast_two_sum would
// break exactness.  Every intended FMA is written as an explicit fma().
#pragma once

#include <math.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define PE_HD __host__ __device__ __forceinline__
#else
#define PE_HD inline
#endif

namespace pe {

struct dd {
    double hi, lo;
};

PE_HD dd two_sum(double a, double b)
{
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}

PE_HD dd fast_two_sum(double a, double b)
{
    double s = a + b;
    double e = b - (s - a);
    return {s, e};
}

PE_HD dd two_prod(double a, double b)
{
    double p = a * b;
    double e = fma(a, b, -p);
    return {p, e};
}

// accurate double-word + double-word
PE_HD dd dw_add(dd x, dd y)
{
    dd s = two_sum(x.hi, y.hi);
    dd t = two_sum(x.lo, y.lo);
    double c = s.lo + t.hi;
    dd v = fast_two_sum(s.hi, c);
    double w = t.lo + v.lo;
    return fast_two_sum(v.hi, w);
}

// sloppy double-word + double-word: |error| <= 4 u^2 (|x| + |y|)
PE_HD dd dw_sum(dd x, dd y)
{
    dd s = two_sum(x.hi, y.hi);
    double c = s.lo + (x.lo + y.lo);
    return fast_two_sum(s.hi, c);
}

// Running sum of double-words (cascaded summation in the manner of Ogita,
// Rump & Oishi's Sum2): the high words go through TwoSum into s, the low
// words and every TwoSum error into one FP64 compensation c; the result is
// FastTwoSum(s, c).  8 instructions per term, and only the add into s is on
// the dependency chain from one term to the next.  Each TwoSum error is at
// most u times the sum of magnitudes S and c adds N of them in FP64, so
// after N terms |error| <= 2 (N+1)^2 u^2 S (tested in rationals); the
// summation uses it for pieces of at most 32 terms (<= 2.7e-29 S).
struct DWAcc {
    double s, c;
};

PE_HD DWAcc dw_acc(dd x) { return {x.hi, x.lo}; }

PE_HD void dw_acc_add(DWAcc &a, dd x)
{
    const dd e = two_sum(a.s, x.hi);
    a.s = e.hi;
    a.c = a.c + (e.lo + x.lo);
}

PE_HD dd dw_acc_get(const DWAcc &a) { return fast_two_sum(a.s, a.c); }

// double-word * double-word with FMA (includes the lo*lo term)
PE_HD dd dw_mul(dd x, dd y)
{
    double ch = x.hi * y.hi;
    double cl1 = fma(x.hi, y.hi, -ch);
    double tl0 = x.lo * y.lo;
    double tl1 = fma(x.hi, y.lo, tl0);
    double cl2 = fma(x.lo, y.hi, tl1);
    double cl3 = cl1 + cl2;
    return fast_two_sum(ch, cl3);
}

// double-word * double with FMA
PE_HD dd dw_mul_d(dd x, double y)
{
    double ch = x.hi * y;
    double cl1 = fma(x.hi, y, -ch);
    double cl3 = fma(x.lo, y, cl1);
    return fast_two_sum(ch, cl3);
}

PE_HD dd dw_neg(dd x) { return {-x.hi, -x.lo}; }

// 1 / y by one Newton-Raphson step from the FP64 reciprocal: e = 1 - y*r0 is
// formed with an exact product (1 - p is exact near 1), then r0 + r0*e is
// renormalized; relative error a few u^2.
PE_HD dd dw_recip(dd y)
{
    double r0 = 1.0 / y.hi;
    double p = y.hi * r0;
    double pe = fma(y.hi, r0, -p);
    double e = 1.0 - p;
    e = e - pe;
    e = fma(-y.lo, r0, e);
    return fast_two_sum(r0, r0 * e);
}

// a*b + c*d for double-words, fused (one part of a complex product).
PE_HD dd dw_dot2(dd a, dd b, dd c, dd d)
{
    double p1 = a.hi * b.hi;
    double e1 = fma(a.hi, b.hi, -p1);
    double p2 = c.hi * d.hi;
    double e2 = fma(c.hi, d.hi, -p2);
    dd s = two_sum(p1, p2);
    double t = fma(a.hi, b.lo, e1);
    t = fma(a.lo, b.hi, t);
    t = fma(c.hi, d.lo, t);
    t = fma(c.lo, d.hi, t);
    t = t + e2;
    t = t + s.lo;
    return fast_two_sum(s.hi, t);
}

// ---------------------------------------------------------------------------
// Arithmetic policies.  A policy supplies the complex type C and the
// operations the evaluation needs; kernels are templated on the policy.
// ---------------------------------------------------------------------------

// complex double-double, fused products
struct ArithDD {
    struct C {
        dd re, im;
    };
    static constexpr int kWords = 4;  // doubles per complex value

    PE_HD static C zero() { return {{0.0, 0.0}, {0.0, 0.0}}; }
    PE_HD static C one() { return {{1.0, 0.0}, {0.0, 0.0}}; }
    PE_HD static C mul(C a, C b)
    {
        return {dw_dot2(a.re, b.re, dw_neg(a.im), b.im), dw_dot2(a.re, b.im, a.im, b.re)};
    }
    PE_HD static C add(C a, C b) { return {dw_add(a.re, b.re), dw_add(a.im, b.im)}; }
    // term of a long sum (sloppy, error relative to the magnitudes)
    PE_HD static C sum(C a, C b) { return {dw_sum(a.re, b.re), dw_sum(a.im, b.im)}; }
    // running sums of many terms (see DWAcc)
    struct Acc {
        DWAcc re, im;
    };
    PE_HD static Acc acc(C a) { return {dw_acc(a.re), dw_acc(a.im)}; }
    PE_HD static void acc_add(Acc &s, C a)
    {
        dw_acc_add(s.re, a.re);
        dw_acc_add(s.im, a.im);
    }
    PE_HD static C acc_get(const Acc &s) { return {dw_acc_get(s.re), dw_acc_get(s.im)}; }
    PE_HD static C neg(C a) { return {dw_neg(a.re), dw_neg(a.im)}; }
    // multiply by a small exact integer held in a double
    PE_HD static C scale(C a, double s) { return {dw_mul_d(a.re, s), dw_mul_d(a.im, s)}; }
    // 1 / b = conj(b) / |b|^2
    PE_HD static C inv(C b)
    {
        dd den = dw_add(dw_mul(b.re, b.re), dw_mul(b.im, b.im));
        dd r = dw_recip(den);
        return {dw_mul(b.re, r), dw_neg(dw_mul(b.im, r))};
    }
    // cheap magnitude for pivot choice
    PE_HD static double mag(C a) { return fabs(a.re.hi) + fabs(a.im.hi); }
};

// complex double-double, textbook product from four double-word products
// and two double-word sums (reference for tests and ablations)
struct ArithDDRef : ArithDD {
    PE_HD static C mul(C a, C b)
    {
        C r;
        r.re = dw_add(dw_mul(a.re, b.re), dw_neg(dw_mul(a.im, b.im)));
        r.im = dw_add(dw_mul(a.re, b.im), dw_mul(a.im, b.re));
        return r;
    }
};

// complex FP64
struct Arith64 {
    struct C {
        double re, im;
    };
    static constexpr int kWords = 2;

    PE_HD static C zero() { return {0.0, 0.0}; }
    PE_HD static C one() { return {1.0, 0.0}; }
    PE_HD static C mul(C a, C b)
    {
        return {fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re)};
    }
    PE_HD static C add(C a, C b) { return {a.re + b.re, a.im + b.im}; }
    PE_HD static C sum(C a, C b) { return add(a, b); }
    using Acc = C;
    PE_HD static Acc acc(C a) { return a; }
    PE_HD static void acc_add(Acc &s, C a) { s = add(s, a); }
    PE_HD static C acc_get(const Acc &s) { return s; }
    PE_HD static C neg(C a) { return {-a.re, -a.im}; }
    PE_HD static C scale(C a, double s) { return {a.re * s, a.im * s}; }
    PE_HD static C inv(C b)
    {
        double den = fma(b.re, b.re, b.im * b.im);
        double r = 1.0 / den;
        return {b.re * r, -b.im * r};
    }
    PE_HD static double mag(C a) { return fabs(a.re) + fabs(a.im); }
};

}  // namespace pe
