// Test-only shim: the library's quad-double arithmetic (qd.hpp), compiled
// for the host with g++ and exposed to the CPU tests through a C interface.
#include "qd.hpp"

using namespace pe;

static qd ld(const double *x) { return {x[0], x[1], x[2], x[3]}; }
static void st(const qd &r, double *o)
{
    o[0] = r.x0;
    o[1] = r.x1;
    o[2] = r.x2;
    o[3] = r.x3;
}

extern "C" {
void qp_add(const double *a, const double *b, double *o) { st(qd_add(ld(a), ld(b)), o); }
void qp_mul(const double *a, const double *b, double *o) { st(qd_mul(ld(a), ld(b)), o); }
void qp_dot2(const double *a, const double *b, const double *c, const double *d, double *o)
{
    st(qd_dot2(ld(a), ld(b), ld(c), ld(d)), o);
}
void qp_mul_d(const double *a, double s, double *o) { st(qd_mul_d(ld(a), s), o); }
// complex product (re, im planes of 4 words each: a[0..3] re, a[4..7] im)
void qp_cmul(const double *a, const double *b, double *o)
{
    ArithQD::C x{ld(a), ld(a + 4)}, y{ld(b), ld(b + 4)};
    ArithQD::C r = ArithQD::mul(x, y);
    st(r.re, o);
    st(r.im, o + 4);
}
}
