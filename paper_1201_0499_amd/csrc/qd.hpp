// Complex quad-double arithmetic: the evaluation one level of precision
// above double-double (the paper's Section 1 cites quad double arithmetic
// beside double double as the way to more accurate path tracking).
//
// A quad-double number is an unevaluated sum x0 + x1 + x2 + x3 of doubles of
// decreasing magnitude.  Every operation here collects the exact or
// first-neglected terms of its result as a short vector of doubles and then
// "distils" the vector: four passes of error-free vector summation from the
// smallest entry up (each pass replaces the entries by their rounded running
// sum and the TwoSum errors, so the exact total never changes), after which
// the first four entries are the result's components.  The terms dropped are
//   - in a sum: nothing (all eight components enter);
//   - in a product: the products x_i y_j with i + j >= 4 and the rounding of
//     the terms of order 3 (x_i y_j with i + j = 3 and the TwoProduct errors
//     of order 2), all below a small multiple of u^4 |x||y|, u = 2^-53;
// so each operation errs by a small multiple of u^4 = 2^-212 relative to the
// magnitudes involved, plus what the distillation leaves after four passes,
// of the same order.  The tests check the evaluation against exact rationals.
//
// Must be compiled with -ffp-contract=off (as dd.hpp); every intended FMA is
// an explicit fma().
#pragma once

#include "dd.hpp"

namespace pe {

struct qd {
    double x0, x1, x2, x3;
};

// four passes of error-free vector summation over e[0..M-1]; e[0..3] then
// hold the components of the total (zero words moved last)
template <int M>
PE_HD qd distill(double (&e)[M])
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double s = e[M - 1];
#pragma unroll
        for (int i = M - 2; i >= j; --i) {
            const dd t = two_sum(e[i], s);
            s = t.hi;
            e[i + 1] = t.lo;
        }
        e[j] = s;
    }
    // after an exact cancellation a leading entry can be zero with the
    // remainder further down: move zero words to the end
    double w[4] = {e[0], e[1], e[2], e[3]};
#pragma unroll
    for (int pass = 0; pass < 3; ++pass)
#pragma unroll
        for (int i = 0; i < 3; ++i)
            if (w[i] == 0.0) {
                w[i] = w[i + 1];
                w[i + 1] = 0.0;
            }
    // the leading entry is the recursively rounded sum, a few ulps off the
    // correctly rounded one; one top-down sweep of FastTwoSum (the words
    // already decrease in magnitude) separates the words
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const dd t = fast_two_sum(w[i], w[i + 1]);
        w[i] = t.hi;
        w[i + 1] = t.lo;
    }
    return {w[0], w[1], w[2], w[3]};
}

PE_HD qd qd_neg(const qd &a) { return {-a.x0, -a.x1, -a.x2, -a.x3}; }

PE_HD qd qd_add(const qd &a, const qd &b)
{
    double e[8] = {a.x0, b.x0, a.x1, b.x1, a.x2, b.x2, a.x3, b.x3};
    return distill<8>(e);
}

// the significant terms of a * b: nine exact leading terms (products and
// TwoProduct errors of order 0..2) written to t, and the order-3 terms
// added into t3
PE_HD void qd_prod_terms(const qd &a, const qd &b, double *t, double &t3)
{
    const dd p00 = two_prod(a.x0, b.x0);
    const dd p01 = two_prod(a.x0, b.x1), p10 = two_prod(a.x1, b.x0);
    const dd p02 = two_prod(a.x0, b.x2), p11 = two_prod(a.x1, b.x1), p20 = two_prod(a.x2, b.x0);
    t[0] = p00.hi;
    t[1] = p00.lo;
    t[2] = p01.hi;
    t[3] = p10.hi;
    t[4] = p01.lo;
    t[5] = p10.lo;
    t[6] = p02.hi;
    t[7] = p11.hi;
    t[8] = p20.hi;
    t3 += fma(a.x0, b.x3, fma(a.x1, b.x2, fma(a.x2, b.x1, a.x3 * b.x0)));
    t3 += p02.lo + p11.lo + p20.lo;
}

PE_HD qd qd_mul(const qd &a, const qd &b)
{
    double e[10];
    double t3 = 0.0;
    qd_prod_terms(a, b, e, t3);
    e[9] = t3;
    return distill<10>(e);
}

// a * b + c * d with one distillation
PE_HD qd qd_dot2(const qd &a, const qd &b, const qd &c, const qd &d)
{
    double e[19];
    double t3 = 0.0;
    qd_prod_terms(a, b, e, t3);
    qd_prod_terms(c, d, e + 9, t3);
    e[18] = t3;
    return distill<19>(e);
}

// a * s for a double s (the small integer exponents of the kernels)
PE_HD qd qd_mul_d(const qd &a, double s)
{
    const dd p0 = two_prod(a.x0, s), p1 = two_prod(a.x1, s), p2 = two_prod(a.x2, s);
    double e[6] = {p0.hi, p0.lo, p1.hi, p1.lo, p2.hi, fma(a.x3, s, p2.lo)};
    return distill<6>(e);
}

// complex quad-double
struct ArithQD {
    struct C {
        qd re, im;
    };
    static constexpr int kWords = 8;

    PE_HD static C zero() { return {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}}; }
    PE_HD static C one() { return {{1.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}}; }
    PE_HD static C mul(const C &a, const C &b)
    {
        return {qd_dot2(a.re, b.re, qd_neg(a.im), b.im), qd_dot2(a.re, b.im, a.im, b.re)};
    }
    PE_HD static C add(const C &a, const C &b) { return {qd_add(a.re, b.re), qd_add(a.im, b.im)}; }
    PE_HD static C sum(const C &a, const C &b) { return add(a, b); }
    using Acc = C;
    PE_HD static Acc acc(const C &a) { return a; }
    PE_HD static void acc_add(Acc &s, const C &a) { s = add(s, a); }
    PE_HD static C acc_get(const Acc &s) { return s; }
    PE_HD static C neg(const C &a) { return {qd_neg(a.re), qd_neg(a.im)}; }
    PE_HD static C scale(const C &a, double s) { return {qd_mul_d(a.re, s), qd_mul_d(a.im, s)}; }
    PE_HD static double mag(const C &a) { return fabs(a.re.x0) + fabs(a.im.x0); }
};

}  // namespace pe
