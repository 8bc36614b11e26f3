// Test-only shim: the library's device arithmetic (dd.hpp) and per-monomial
// routine (monomial.hpp), compiled for the host with g++ and exposed to the
// CPU tests through a small C interface.
#include <cstdint>

#include "dd.hpp"
#include "monomial.hpp"

using namespace pe;

extern "C" {

void ap_two_sum(double a, double b, double *o) { dd r = two_sum(a, b); o[0] = r.hi; o[1] = r.lo; }
void ap_two_prod(double a, double b, double *o) { dd r = two_prod(a, b); o[0] = r.hi; o[1] = r.lo; }
void ap_dw_add(const double *x, const double *y, double *o)
{
    dd r = dw_add({x[0], x[1]}, {y[0], y[1]});
    o[0] = r.hi;
    o[1] = r.lo;
}
void ap_dw_sum(const double *x, const double *y, double *o)
{
    dd r = dw_sum({x[0], x[1]}, {y[0], y[1]});
    o[0] = r.hi;
    o[1] = r.lo;
}
void ap_dw_mul(const double *x, const double *y, double *o)
{
    dd r = dw_mul({x[0], x[1]}, {y[0], y[1]});
    o[0] = r.hi;
    o[1] = r.lo;
}
void ap_dw_mul_d(const double *x, double y, double *o)
{
    dd r = dw_mul_d({x[0], x[1]}, y);
    o[0] = r.hi;
    o[1] = r.lo;
}

// cascaded sum of n double-words x[2i], x[2i+1]
void ap_dw_acc(const double *x, int n, double *o)
{
    DWAcc a = dw_acc({x[0], x[1]});
    for (int i = 1; i < n; ++i) dw_acc_add(a, {x[2 * i], x[2 * i + 1]});
    dd r = dw_acc_get(a);
    o[0] = r.hi;
    o[1] = r.lo;
}

// complex dd as 4 doubles (re_hi, re_lo, im_hi, im_lo)
static ArithDD::C ld(const double *a) { return {{a[0], a[1]}, {a[2], a[3]}}; }
static void st(double *o, ArithDD::C v)
{
    o[0] = v.re.hi;
    o[1] = v.re.lo;
    o[2] = v.im.hi;
    o[3] = v.im.lo;
}
void ap_cmul(const double *a, const double *b, double *o) { st(o, ArithDD::mul(ld(a), ld(b))); }
void ap_cmul_ref(const double *a, const double *b, double *o) { st(o, ArithDDRef::mul(ld(a), ld(b))); }
void ap_cadd(const double *a, const double *b, double *o) { st(o, ArithDD::add(ld(a), ld(b))); }

}  // extern "C"

// ---- operation counting -------------------------------------------------
struct ArithCount {
    struct C {
        double v;
    };
    static inline long muls = 0, adds = 0, scales = 0;
    static C zero() { return {0}; }
    static C one() { return {1}; }
    static C mul(C a, C b)
    {
        ++muls;
        return {a.v * b.v};
    }
    static C add(C a, C b)
    {
        ++adds;
        return {a.v + b.v};
    }
    static C sum(C a, C b) { return add(a, b); }
    static C scale(C a, double s)
    {
        ++scales;
        return {a.v * s};
    }
};

template <int CC>
static void count_cc(long *out)
{
    using C = ArithCount::C;
    ArithCount::muls = ArithCount::adds = ArithCount::scales = 0;
    double xs[CC];
    for (int t = 0; t < CC; ++t) xs[t] = (t % 3 == 0) ? 0.5 : (t % 3 == 1 ? 2.0 : 4.0);
    auto x = [&](int t) { return C{xs[t]}; };
    C lp[CC], P;
    speelpenning<ArithCount, CC>(x, lp, P);
    out[0] = ArithCount::muls;  // Speelpenning partials + full product
    ArithCount::muls = 0;
    C cf = common_factor<ArithCount, CC>(x);
    out[1] = ArithCount::muls;  // common factor
    ArithCount::muls = 0;
    auto ae = [](int) { return 1.0; };
    C D[CC], V;
    monomial_terms<ArithCount, CC>(x, cf, ae, C{1.0}, SoloGroup{}, D, V);
    out[2] = ArithCount::muls;   // everything after the common factor
    out[3] = ArithCount::scales; // exponent scalings
    // values: lp[t] = prod_{t' != t} x_t', P = prod x
    double prod = 1.0;
    for (int t = 0; t < CC; ++t) prod *= xs[t];
    int ok = (P.v == prod);
    for (int t = 0; t < CC; ++t) ok &= (lp[t].v * xs[t] == prod);
    out[4] = ok;
}

extern "C" int ap_count_ops(int cc, long *out)
{
    switch (cc) {
    case 1: count_cc<1>(out); return 0;
    case 2: count_cc<2>(out); return 0;
    case 3: count_cc<3>(out); return 0;
    case 4: count_cc<4>(out); return 0;
    case 5: count_cc<5>(out); return 0;
    case 8: count_cc<8>(out); return 0;
    case 9: count_cc<9>(out); return 0;
    case 16: count_cc<16>(out); return 0;
    case 32: count_cc<32>(out); return 0;
    }
    return 1;
}
