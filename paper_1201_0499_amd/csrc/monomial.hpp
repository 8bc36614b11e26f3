// Per-lane work on one monomial: common factor, Speelpenning product with
// forward and backward partial products, coefficient and exponent scaling.
//
// A monomial c * x_{i_1}^{a_1} ... x_{i_k}^{a_k} (Section 2, stages 1 and 2)
// is evaluated with all k partial derivatives as
//
//   CF  = x_{i_1}^{a_1-1} ... x_{i_k}^{a_k-1}          (common factor, 3.1)
//   S_j = prod_{l != j} x_{i_l}                        (Speelpenning, 3.2)
//   df/dx_{i_j} = c * a_j * CF * S_j                   (3.2 and 3.3)
//   value       = c * CF * S_k * x_{i_k}               (3.2)
//
// Its k variables are split over a group of L lanes, CC consecutive
// variables per lane.  Each lane forms the Speelpenning partials of its own
// CC variables (3CC-6 products, the forward/backward scheme of Section 3.2:
// forward products stored, one running backward product), the product P of
// its CC variables and the product cf of its CC common-factor entries.  The
// group then forms, with a butterfly over its lanes, each lane's exclusive
// product E = prod over the other lanes of cf*P.  The partial with respect
// to the lane's t-th variable is w * lp[t] with w = c * cf * E (the full
// common factor times the other lanes' variables times the coefficient),
// and the value is w * P.  With L = 1 this is the paper's single-thread
// scheme.
//
// Variables are read through an accessor (on the GPU: from the LDS power
// table, as the paper reads them from shared memory) so that they need not
// stay in registers.  Everything here is __host__ __device__ and templated
// on the arithmetic policy, so the same code runs in the kernels and, on the
// host, under an operation-counting policy in the tests.
#pragma once

#include "dd.hpp"

namespace pe {

// Speelpenning product of x(0..CC): lp[t] = prod_{t' != t} x(t') and
// P = prod x.  CC >= 3 uses the forward/backward scheme (3CC-6 products for
// the partials, one more for P).
template <class A, int CC, class X>
PE_HD void speelpenning(const X &x, typename A::C (&lp)[CC], typename A::C &P)
{
    using C = typename A::C;
    if constexpr (CC == 1) {
        lp[0] = A::one();
        P = x(0);
    } else if constexpr (CC == 2) {
        lp[0] = x(1);
        lp[1] = x(0);
        P = A::mul(lp[1], lp[0]);
    } else {
        // forward products: lp[r] = x_0 ... x_{r-1}, r = 1 .. CC-1
        lp[1] = x(0);
#pragma unroll
        for (int r = 2; r < CC; ++r) lp[r] = A::mul(lp[r - 1], x(r - 1));
        // lp[CC-1] is the partial with respect to x_{CC-1}
        C Q = x(CC - 1);
        P = A::mul(lp[CC - 1], Q);
        // backward product Q = x_{CC-1} x_{CC-2} ... combined with forward ones
        lp[CC - 2] = A::mul(lp[CC - 2], Q);
#pragma unroll
        for (int r = CC - 3; r >= 1; --r) {
            Q = A::mul(Q, x(r + 1));
            lp[r] = A::mul(lp[r], Q);
        }
        lp[0] = A::mul(Q, x(1));
    }
}

// Lane-group exchange for L = 1 (and on the host): a single lane.
struct SoloGroup {
    template <class A>
    PE_HD void combine(const typename A::C &, const typename A::C &, typename A::C &,
                       bool &have_E) const
    {
        have_E = false;
    }
};

// The terms of one lane given its common-factor product cf: D[t] =
// c a_t CF S_t for its CC variables (aexp(t) = a_t) and the monomial value V
// (meaningful on every lane; the caller keeps one).
template <class A, int CC, class X, class Exps, class Group>
PE_HD void monomial_terms(const X &x, typename A::C cf, const Exps &aexp, typename A::C coef,
                          const Group &grp, typename A::C (&D)[CC], typename A::C &V)
{
    using C = typename A::C;
    C P;
    speelpenning<A, CC>(x, D, P);  // D holds the partials lp[t] until scaled
    C E;
    bool have_E;
    grp.template combine<A>(cf, P, E, have_E);
    C w = A::mul(cf, coef);
    if (have_E) w = A::mul(w, E);
#pragma unroll
    for (int t = 0; t < CC; ++t) D[t] = A::scale(A::mul(w, D[t]), aexp(t));
    V = A::mul(w, P);
}

// Product of common-factor entries z(0..CC) (CC-1 products).
template <class A, int CC, class Z>
PE_HD typename A::C common_factor(const Z &z)
{
    typename A::C cf = z(0);
#pragma unroll
    for (int t = 1; t < CC; ++t) cf = A::mul(cf, z(t));
    return cf;
}

}  // namespace pe
