/*
 * ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU evaluator of a sparse polynomial system f = (C, A) and
 * its Jacobian, in complex double-double (dd) and in complex FP64, plus a
 * plain dd Newton corrector.  It exists to check the GPU library; only the
 * tests, the package's smoke entry and the CPU-baseline leg of the bench may
 * load it.  It shares no code with the GPU path.
 *
 * What it computes is the definition in Section 2, equation (1), of the
 * paper (Verschelde & Yoffe, "Evaluating polynomials in several variables and
 * their derivatives on a GPU computing processor"):
 *
 *     f_p(x)     = sum_{s in p} c_s * prod_j x_{i_j}^{a_j}
 *     df_p/dx_i  = sum_{s in p, i in supp s} c_s * a_i * x_i^{a_i - 1}
 *                                              * prod_{j: i_j != i} x_{i_j}^{a_j}
 *
 * written out term by term: every power is a chain of plain multiplications
 * starting from the coefficient, every partial derivative is its own product
 * (O(k^2) work per monomial), and sums run left to right in monomial order.
 * There is no power table, no common factor and no Speelpenning product here.
 *
 * dd arithmetic, from published error-free transformations, without FMA:
 *   - TwoSum (Knuth, TAOCP vol. 2, 4.2.2; Moller 1965),
 *   - FastTwoSum (Dekker 1971),
 *   - TwoProduct via Veltkamp's split (Dekker 1971),
 *   - accurate double-word + double-word sum and the double-word product
 *     without FMA as analysed by Joldes, Muller & Popescu, ACM TOMS 44(2),
 *     2017 ("AccurateDWPlusDW", "DWTimesDW1").
 * Complex products use the textbook four-product form.  Build with
 * -ffp-contract=off so the compiler fuses no multiply-add.
 *
 * Layouts (all row-major C arrays of doubles, one array per plane
 * re_hi, re_lo, im_hi, im_lo; FP64 entry points use re_hi/im_hi only):
 *   x : [n_points][n_vars]
 *   f : [n_points][n_polys]
 *   J : [n_points][n_vars][n_polys]   (column-major Jacobian per point:
 *                                      entry (p, i) at i*n_polys + p)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double hi, lo; } odd;
typedef struct { odd re, im; } ocdd;
typedef struct { double re, im; } oc64;

/* ----------------------------------------------------------------------- */
/* error-free transformations                                               */
/* ----------------------------------------------------------------------- */

static odd o_two_sum(double a, double b)
{
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    odd r = {s, e};
    return r;
}

static odd o_fast_two_sum(double a, double b) /* requires |a| >= |b| or a == 0 */
{
    double s = a + b;
    double e = b - (s - a);
    odd r = {s, e};
    return r;
}

static void o_split(double a, double *h, double *l) /* Veltkamp, C = 2^27 + 1 */
{
    double c = 134217729.0 * a;
    double big = c - a;
    *h = c - big;
    *l = a - *h;
}

static odd o_two_prod(double a, double b)
{
    double p = a * b;
    double ah, al, bh, bl;
    o_split(a, &ah, &al);
    o_split(b, &bh, &bl);
    double e = ((ah * bh - p) + ah * bl + al * bh) + al * bl;
    odd r = {p, e};
    return r;
}

/* ----------------------------------------------------------------------- */
/* double-word arithmetic                                                   */
/* ----------------------------------------------------------------------- */

static odd o_add(odd x, odd y) /* AccurateDWPlusDW */
{
    odd s = o_two_sum(x.hi, y.hi);
    odd t = o_two_sum(x.lo, y.lo);
    double c = s.lo + t.hi;
    odd v = o_fast_two_sum(s.hi, c);
    double w = t.lo + v.lo;
    return o_fast_two_sum(v.hi, w);
}

static odd o_neg(odd x)
{
    odd r = {-x.hi, -x.lo};
    return r;
}

static odd o_mul(odd x, odd y) /* DWTimesDW1 (no FMA) */
{
    odd c = o_two_prod(x.hi, y.hi);
    double t1 = x.hi * y.lo;
    double t2 = x.lo * y.hi;
    double c2 = t1 + t2;
    double c3 = c.lo + c2;
    return o_fast_two_sum(c.hi, c3);
}

static odd o_from(double a)
{
    odd r = {a, 0.0};
    return r;
}

/* x / y by long division with two correction steps */
static odd o_div(odd x, odd y)
{
    double q1 = x.hi / y.hi;
    odd r = o_add(x, o_neg(o_mul(y, o_from(q1))));
    double q2 = r.hi / y.hi;
    r = o_add(r, o_neg(o_mul(y, o_from(q2))));
    double q3 = r.hi / y.hi;
    odd q = o_fast_two_sum(q1, q2);
    return o_add(q, o_from(q3));
}

/* complex double-double */
static ocdd c_add(ocdd a, ocdd b)
{
    ocdd r = {o_add(a.re, b.re), o_add(a.im, b.im)};
    return r;
}

static ocdd c_sub(ocdd a, ocdd b)
{
    ocdd r = {o_add(a.re, o_neg(b.re)), o_add(a.im, o_neg(b.im))};
    return r;
}

static ocdd c_mul(ocdd a, ocdd b)
{
    ocdd r;
    r.re = o_add(o_mul(a.re, b.re), o_neg(o_mul(a.im, b.im)));
    r.im = o_add(o_mul(a.re, b.im), o_mul(a.im, b.re));
    return r;
}

static ocdd c_scale(ocdd a, double s)
{
    ocdd r = {o_mul(a.re, o_from(s)), o_mul(a.im, o_from(s))};
    return r;
}

static ocdd c_div(ocdd a, ocdd b) /* a * conj(b) / |b|^2 */
{
    odd den = o_add(o_mul(b.re, b.re), o_mul(b.im, b.im));
    ocdd bc = {b.re, o_neg(b.im)};
    ocdd num = c_mul(a, bc);
    ocdd r = {o_div(num.re, den), o_div(num.im, den)};
    return r;
}

static const ocdd C_ZERO = {{0.0, 0.0}, {0.0, 0.0}};

/* complex FP64 */
static oc64 d_add(oc64 a, oc64 b)
{
    oc64 r = {a.re + b.re, a.im + b.im};
    return r;
}

static oc64 d_mul(oc64 a, oc64 b)
{
    oc64 r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return r;
}

/* ----------------------------------------------------------------------- */
/* exported primitives (for the oracle's own tests)                         */
/* ----------------------------------------------------------------------- */

void orc_two_sum(double a, double b, double *s, double *e)
{
    odd r = o_two_sum(a, b);
    *s = r.hi;
    *e = r.lo;
}

void orc_two_prod(double a, double b, double *p, double *e)
{
    odd r = o_two_prod(a, b);
    *p = r.hi;
    *e = r.lo;
}

void orc_dd_add(double xh, double xl, double yh, double yl, double *zh, double *zl)
{
    odd x = {xh, xl}, y = {yh, yl};
    odd z = o_add(x, y);
    *zh = z.hi;
    *zl = z.lo;
}

void orc_dd_mul(double xh, double xl, double yh, double yl, double *zh, double *zl)
{
    odd x = {xh, xl}, y = {yh, yl};
    odd z = o_mul(x, y);
    *zh = z.hi;
    *zl = z.lo;
}

void orc_dd_div(double xh, double xl, double yh, double yl, double *zh, double *zl)
{
    odd x = {xh, xl}, y = {yh, yl};
    odd z = o_div(x, y);
    *zh = z.hi;
    *zl = z.lo;
}

/* ----------------------------------------------------------------------- */
/* the definition, in complex dd                                            */
/* ----------------------------------------------------------------------- */

static ocdd load_cdd(const double *const pl[4], int64_t i)
{
    ocdd r = {{pl[0][i], pl[1][i]}, {pl[2][i], pl[3][i]}};
    return r;
}

static void store_cdd(double *const pl[4], int64_t i, ocdd v)
{
    pl[0][i] = v.re.hi;
    pl[1][i] = v.re.lo;
    pl[2][i] = v.im.hi;
    pl[3][i] = v.im.lo;
}

/*
 * One point x (n_vars entries) -> f (n_polys) and, if J_col != NULL, the
 * Jacobian as an array J_col[i*n_polys + p].  Only polynomials listed in
 * `polys` (n_sel of them) are evaluated; the others are left untouched.
 */
static void eval_point_dd(int32_t n_vars, int32_t n_polys,
                          const int64_t *poly_start, const int64_t *mono_start,
                          const int32_t *pos, const int32_t *expo,
                          const double *const coef[4], const ocdd *x,
                          ocdd *f, ocdd *J_col, const int32_t *polys, int32_t n_sel)
{
    for (int32_t t = 0; t < n_sel; ++t) {
        int32_t p = polys[t];
        ocdd fp = C_ZERO;
        if (J_col)
            for (int32_t i = 0; i < n_vars; ++i)
                J_col[(int64_t)i * n_polys + p] = C_ZERO;
        for (int64_t s = poly_start[p]; s < poly_start[p + 1]; ++s) {
            int64_t b = mono_start[s], e = mono_start[s + 1];
            ocdd c = load_cdd(coef, s);
            /* value: c * x_{i_1}^{a_1} * ... * x_{i_k}^{a_k} */
            ocdd v = c;
            for (int64_t j = b; j < e; ++j)
                for (int32_t r = 0; r < expo[j]; ++r)
                    v = c_mul(v, x[pos[j]]);
            fp = c_add(fp, v);
            if (!J_col)
                continue;
            /* each partial derivative as its own product */
            for (int64_t j = b; j < e; ++j) {
                ocdd d = c_scale(c, (double)expo[j]);
                for (int64_t l = b; l < e; ++l) {
                    int32_t times = expo[l] - (l == j ? 1 : 0);
                    for (int32_t r = 0; r < times; ++r)
                        d = c_mul(d, x[pos[l]]);
                }
                int64_t at = (int64_t)pos[j] * n_polys + p;
                J_col[at] = c_add(J_col[at], d);
            }
        }
        f[p] = fp;
    }
}

static int32_t *all_polys(int32_t n_polys)
{
    int32_t *sel = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_polys > 0 ? n_polys : 1));
    for (int32_t p = 0; p < n_polys; ++p)
        sel[p] = p;
    return sel;
}

int orc_eval_dd(int32_t n_vars, int32_t n_polys, const int64_t *poly_start,
                const int64_t *mono_start, const int32_t *pos, const int32_t *expo,
                const double *const coef[4], int64_t n_points, const double *const x[4],
                double *const f[4], double *const J[4], const int32_t *polys, int32_t n_sel)
{
    int32_t *own = NULL;
    if (!polys) {
        own = all_polys(n_polys);
        polys = own;
        n_sel = n_polys;
    }
    ocdd *xp = (ocdd *)malloc(sizeof(ocdd) * (size_t)n_vars);
    ocdd *fp = (ocdd *)malloc(sizeof(ocdd) * (size_t)n_polys);
    ocdd *Jp = J ? (ocdd *)malloc(sizeof(ocdd) * (size_t)n_vars * (size_t)n_polys) : NULL;
    for (int64_t q = 0; q < n_points; ++q) {
        for (int32_t i = 0; i < n_vars; ++i)
            xp[i] = load_cdd(x, q * n_vars + i);
        eval_point_dd(n_vars, n_polys, poly_start, mono_start, pos, expo, coef, xp, fp, Jp,
                      polys, n_sel);
        for (int32_t t = 0; t < n_sel; ++t) {
            int32_t p = polys[t];
            store_cdd(f, q * n_polys + p, fp[p]);
            if (J)
                for (int32_t i = 0; i < n_vars; ++i) {
                    int64_t at = (int64_t)i * n_polys + p;
                    store_cdd(J, q * (int64_t)n_vars * n_polys + at, Jp[at]);
                }
        }
    }
    free(xp);
    free(fp);
    free(Jp);
    free(own);
    return 0;
}

/* ----------------------------------------------------------------------- */
/* the definition, in complex FP64                                          */
/* ----------------------------------------------------------------------- */

int orc_eval_f64(int32_t n_vars, int32_t n_polys, const int64_t *poly_start,
                 const int64_t *mono_start, const int32_t *pos, const int32_t *expo,
                 const double *coef_re, const double *coef_im, int64_t n_points,
                 const double *x_re, const double *x_im, double *f_re, double *f_im,
                 double *J_re, double *J_im, const int32_t *polys, int32_t n_sel)
{
    int32_t *own = NULL;
    if (!polys) {
        own = all_polys(n_polys);
        polys = own;
        n_sel = n_polys;
    }
    for (int64_t q = 0; q < n_points; ++q) {
        const double *xr = x_re + q * n_vars, *xi = x_im + q * n_vars;
        for (int32_t t = 0; t < n_sel; ++t) {
            int32_t p = polys[t];
            oc64 fp = {0.0, 0.0};
            if (J_re)
                for (int32_t i = 0; i < n_vars; ++i) {
                    int64_t at = q * (int64_t)n_vars * n_polys + (int64_t)i * n_polys + p;
                    J_re[at] = 0.0;
                    J_im[at] = 0.0;
                }
            for (int64_t s = poly_start[p]; s < poly_start[p + 1]; ++s) {
                int64_t b = mono_start[s], e = mono_start[s + 1];
                oc64 c = {coef_re[s], coef_im[s]};
                oc64 v = c;
                for (int64_t j = b; j < e; ++j)
                    for (int32_t r = 0; r < expo[j]; ++r) {
                        oc64 xv = {xr[pos[j]], xi[pos[j]]};
                        v = d_mul(v, xv);
                    }
                fp = d_add(fp, v);
                if (!J_re)
                    continue;
                for (int64_t j = b; j < e; ++j) {
                    oc64 d = {c.re * (double)expo[j], c.im * (double)expo[j]};
                    for (int64_t l = b; l < e; ++l) {
                        int32_t times = expo[l] - (l == j ? 1 : 0);
                        for (int32_t r = 0; r < times; ++r) {
                            oc64 xv = {xr[pos[l]], xi[pos[l]]};
                            d = d_mul(d, xv);
                        }
                    }
                    int64_t at = q * (int64_t)n_vars * n_polys + (int64_t)pos[j] * n_polys + p;
                    J_re[at] += d.re;
                    J_im[at] += d.im;
                }
            }
            f_re[q * n_polys + p] = fp.re;
            f_im[q * n_polys + p] = fp.im;
        }
    }
    free(own);
    return 0;
}

/* ----------------------------------------------------------------------- */
/* magnitude scales for a condition-scaled error metric                     */
/*   Sf[p]     = sum_s |c_s| |x^{a_s}|                                      */
/*   SJ[i][p]  = sum_{s: i in supp} |c_s| a_i |x_i|^{a_i-1} prod_{l!=i} |x_l|^{a_l}  */
/* ----------------------------------------------------------------------- */

int orc_scales(int32_t n_vars, int32_t n_polys, const int64_t *poly_start,
               const int64_t *mono_start, const int32_t *pos, const int32_t *expo,
               const double *coef_re, const double *coef_im, int64_t n_points,
               const double *x_re, const double *x_im, double *Sf, double *SJ,
               const int32_t *polys, int32_t n_sel)
{
    int32_t *own = NULL;
    if (!polys) {
        own = all_polys(n_polys);
        polys = own;
        n_sel = n_polys;
    }
    double *ax = (double *)malloc(sizeof(double) * (size_t)n_vars);
    for (int64_t q = 0; q < n_points; ++q) {
        for (int32_t i = 0; i < n_vars; ++i)
            ax[i] = hypot(x_re[q * n_vars + i], x_im[q * n_vars + i]);
        for (int32_t t = 0; t < n_sel; ++t) {
            int32_t p = polys[t];
            double sf = 0.0;
            if (SJ)
                for (int32_t i = 0; i < n_vars; ++i)
                    SJ[q * (int64_t)n_vars * n_polys + (int64_t)i * n_polys + p] = 0.0;
            for (int64_t s = poly_start[p]; s < poly_start[p + 1]; ++s) {
                int64_t b = mono_start[s], e = mono_start[s + 1];
                double c = hypot(coef_re[s], coef_im[s]);
                double v = c;
                for (int64_t j = b; j < e; ++j)
                    v *= pow(ax[pos[j]], (double)expo[j]);
                sf += v;
                if (!SJ)
                    continue;
                for (int64_t j = b; j < e; ++j) {
                    double d = c * (double)expo[j];
                    for (int64_t l = b; l < e; ++l)
                        d *= pow(ax[pos[l]], (double)(expo[l] - (l == j ? 1 : 0)));
                    SJ[q * (int64_t)n_vars * n_polys + (int64_t)pos[j] * n_polys + p] += d;
                }
            }
            Sf[q * n_polys + p] = sf;
        }
    }
    free(ax);
    free(own);
    return 0;
}

/* ----------------------------------------------------------------------- */
/* dense complex dd linear solve: Gaussian elimination, partial pivoting    */
/* A column-major n x n (entry (r, c) at c*n + r), b length n; both are     */
/* overwritten.  Returns 0, or 2 if a pivot is exactly zero, 3 non-finite.  */
/* ----------------------------------------------------------------------- */

static double c_mag(ocdd a)
{
    return hypot(a.re.hi, a.im.hi);
}

static int solve_dd(int32_t n, ocdd *A, ocdd *b, ocdd *x)
{
    for (int32_t c = 0; c < n; ++c) {
        int32_t piv = c;
        double best = c_mag(A[(int64_t)c * n + c]);
        for (int32_t r = c + 1; r < n; ++r) {
            double m = c_mag(A[(int64_t)c * n + r]);
            if (m > best) {
                best = m;
                piv = r;
            }
        }
        if (!(best == best) || isinf(best))
            return 3;
        if (best == 0.0)
            return 2;
        if (piv != c) {
            for (int32_t cc = 0; cc < n; ++cc) {
                ocdd t = A[(int64_t)cc * n + c];
                A[(int64_t)cc * n + c] = A[(int64_t)cc * n + piv];
                A[(int64_t)cc * n + piv] = t;
            }
            ocdd t = b[c];
            b[c] = b[piv];
            b[piv] = t;
        }
        ocdd d = A[(int64_t)c * n + c];
        for (int32_t r = c + 1; r < n; ++r) {
            ocdd l = c_div(A[(int64_t)c * n + r], d);
            for (int32_t cc = c + 1; cc < n; ++cc)
                A[(int64_t)cc * n + r] = c_sub(A[(int64_t)cc * n + r], c_mul(l, A[(int64_t)cc * n + c]));
            b[r] = c_sub(b[r], c_mul(l, b[c]));
        }
    }
    for (int32_t r = n - 1; r >= 0; --r) {
        ocdd s = b[r];
        for (int32_t cc = r + 1; cc < n; ++cc)
            s = c_sub(s, c_mul(A[(int64_t)cc * n + r], x[cc]));
        x[r] = c_div(s, A[(int64_t)r * n + r]);
    }
    return 0;
}

int orc_solve_dd(int32_t n, double *const A[4], double *const b[4], double *const x[4])
{
    ocdd *Am = (ocdd *)malloc(sizeof(ocdd) * (size_t)n * (size_t)n);
    ocdd *bm = (ocdd *)malloc(sizeof(ocdd) * (size_t)n);
    ocdd *xm = (ocdd *)malloc(sizeof(ocdd) * (size_t)n);
    for (int64_t i = 0; i < (int64_t)n * n; ++i)
        Am[i] = load_cdd((const double *const *)A, i);
    for (int32_t i = 0; i < n; ++i)
        bm[i] = load_cdd((const double *const *)b, i);
    int st = solve_dd(n, Am, bm, xm);
    if (st == 0)
        for (int32_t i = 0; i < n; ++i)
            store_cdd(x, i, xm[i]);
    free(Am);
    free(bm);
    free(xm);
    return st;
}

/* ----------------------------------------------------------------------- */
/* plain dd Newton: x <- x - J(x)^{-1} f(x) until max_p |f_p(x)| < tol       */
/* Square systems only.  Per start: status 0 converged, 1 max_iter reached, */
/* 2 zero pivot, 3 non-finite.  res_out = max_p |f_p| at the returned x,    */
/* iters_out = number of updates applied.                                   */
/* ----------------------------------------------------------------------- */

int orc_newton_dd(int32_t n, const int64_t *poly_start, const int64_t *mono_start,
                  const int32_t *pos, const int32_t *expo, const double *const coef[4],
                  int64_t n_starts, double *const x[4], double tol, int32_t max_iter,
                  double *res_out, int32_t *iters_out, int32_t *status_out)
{
    int32_t *sel = all_polys(n);
    ocdd *xp = (ocdd *)malloc(sizeof(ocdd) * (size_t)n);
    ocdd *fp = (ocdd *)malloc(sizeof(ocdd) * (size_t)n);
    ocdd *Jp = (ocdd *)malloc(sizeof(ocdd) * (size_t)n * (size_t)n);
    ocdd *dx = (ocdd *)malloc(sizeof(ocdd) * (size_t)n);
    int any_bad = 0;
    for (int64_t q = 0; q < n_starts; ++q) {
        for (int32_t i = 0; i < n; ++i)
            xp[i] = load_cdd((const double *const *)x, q * n + i);
        int32_t status = 1, it = 0;
        double res = 0.0;
        for (;;) {
            eval_point_dd(n, n, poly_start, mono_start, pos, expo, coef, xp, fp, Jp, sel, n);
            res = 0.0;
            int finite = 1;
            for (int32_t p = 0; p < n; ++p) {
                double m = c_mag(fp[p]);
                if (!(m == m) || isinf(m))
                    finite = 0;
                if (m > res)
                    res = m;
            }
            if (!finite) {
                status = 3;
                break;
            }
            if (res < tol) {
                status = 0;
                break;
            }
            if (it >= max_iter) {
                status = 1;
                break;
            }
            int st = solve_dd(n, Jp, fp, dx);
            if (st) {
                status = st;
                break;
            }
            for (int32_t i = 0; i < n; ++i)
                xp[i] = c_sub(xp[i], dx[i]);
            ++it;
        }
        for (int32_t i = 0; i < n; ++i)
            store_cdd(x, q * n + i, xp[i]);
        res_out[q] = res;
        iters_out[q] = it;
        status_out[q] = status;
        if (status)
            any_bad = 1;
    }
    free(sel);
    free(xp);
    free(fp);
    free(Jp);
    free(dx);
    return any_bad;
}

/* ----------------------------------------------------------------------- */
/* fast mode: the CPU throughput baseline                                   */
/*                                                                          */
/* The same f and J as orc_eval_dd, by the paper's three stages (Section 2) */
/* instead of term-by-term products: per point a table of the powers        */
/* x_i^e, e = 0..d (Section 3.1, first stage); per monomial the common      */
/* factor prod_j x_{i_j}^{a_j - 1} from the table (Section 3.1), every      */
/* partial of the product y_1 ... y_k of its variables as a prefix product  */
/* y_1 ... y_{j-1} times a suffix product y_{j+1} ... y_k (Speelpenning's   */
/* forward and backward products, Section 3.2), and the coefficient and     */
/* exponent scaling c * a_j * CF * partial_j (Sections 3.2 and 3.3).  Sums  */
/* run left to right in monomial order, as above.  Same dd arithmetic as    */
/* the definitional evaluator (no FMA).  OpenMP threads take (point,        */
/* polynomial) pairs; every pair writes its own outputs, so results do not  */
/* depend on the number of threads.  Used only to time the CPU and checked  */
/* against orc_eval_dd by the tests.                                        */
/* ----------------------------------------------------------------------- */

#ifdef _OPENMP
#include <omp.h>
#endif

static const ocdd C_ONE = {{1.0, 0.0}, {0.0, 0.0}};

int orc_eval_dd_fast(int32_t n_vars, int32_t n_polys, const int64_t *poly_start,
                     const int64_t *mono_start, const int32_t *pos, const int32_t *expo,
                     const double *const coef[4], int64_t n_points, const double *const x[4],
                     double *const f[4], double *const J[4], const int32_t *polys,
                     int32_t n_sel, int32_t n_threads, int32_t *threads_used)
{
    int32_t *own = NULL;
    if (!polys) {
        own = all_polys(n_polys);
        polys = own;
        n_sel = n_polys;
    }
    int64_t n_monos = poly_start[n_polys];
    int32_t d = 1, kmax = 1;
    for (int64_t s = 0; s < n_monos; ++s) {
        int32_t k = (int32_t)(mono_start[s + 1] - mono_start[s]);
        if (k > kmax)
            kmax = k;
        for (int64_t j = mono_start[s]; j < mono_start[s + 1]; ++j)
            if (expo[j] > d)
                d = expo[j];
    }
    /* pw[(q * (d + 1) + e) * n_vars + i] = x_i^e at point q */
    ocdd *pw = (ocdd *)malloc(sizeof(ocdd) * (size_t)(n_points > 0 ? n_points : 1) *
                              (size_t)(d + 1) * (size_t)n_vars);
    int used = 1;
#ifdef _OPENMP
    if (n_threads <= 0)
        n_threads = omp_get_max_threads();
#else
    n_threads = 1;
#endif
#pragma omp parallel num_threads(n_threads)
    {
        ocdd *pre = (ocdd *)malloc(sizeof(ocdd) * (size_t)(kmax + 1));
        ocdd *suf = (ocdd *)malloc(sizeof(ocdd) * (size_t)(kmax + 1));
        ocdd *yv = (ocdd *)malloc(sizeof(ocdd) * (size_t)(kmax + 1));
#ifdef _OPENMP
#pragma omp single
        used = omp_get_num_threads();
#endif
#pragma omp for schedule(static)
        for (int64_t t = 0; t < n_points * (int64_t)n_vars; ++t) {
            int64_t q = t / n_vars;
            int32_t i = (int32_t)(t % n_vars);
            ocdd xi = load_cdd(x, t);
            ocdd *col = pw + q * (int64_t)(d + 1) * n_vars;
            col[i] = C_ONE;
            col[n_vars + i] = xi;
            for (int32_t e = 2; e <= d; ++e)
                col[(int64_t)e * n_vars + i] = c_mul(col[(int64_t)(e - 1) * n_vars + i], xi);
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < n_points * (int64_t)n_sel; ++t) {
            int64_t q = t / n_sel;
            int32_t p = polys[t % n_sel];
            const ocdd *tab = pw + q * (int64_t)(d + 1) * n_vars;
            int64_t jbase = q * (int64_t)n_vars * n_polys;
            if (J)
                for (int32_t i = 0; i < n_vars; ++i)
                    store_cdd(J, jbase + (int64_t)i * n_polys + p, C_ZERO);
            ocdd fp = C_ZERO;
            for (int64_t s = poly_start[p]; s < poly_start[p + 1]; ++s) {
                int64_t b = mono_start[s];
                int32_t k = (int32_t)(mono_start[s + 1] - b);
                ocdd c = load_cdd(coef, s);
                if (k == 0) {
                    fp = c_add(fp, c);
                    continue;
                }
                /* common factor times the coefficient */
                ocdd w = c;
                for (int32_t j = 0; j < k; ++j) {
                    yv[j] = tab[n_vars + pos[b + j]];
                    if (expo[b + j] > 1)
                        w = c_mul(w, tab[(int64_t)(expo[b + j] - 1) * n_vars + pos[b + j]]);
                }
                /* prefix products pre[j] = y_0 ... y_{j-1}, suffix products
                   suf[j] = y_j ... y_{k-1} */
                pre[0] = C_ONE;
                pre[1] = yv[0];
                for (int32_t j = 2; j <= k; ++j)
                    pre[j] = c_mul(pre[j - 1], yv[j - 1]);
                fp = c_add(fp, c_mul(w, pre[k]));
                if (!J)
                    continue;
                suf[k] = C_ONE;
                suf[k - 1] = yv[k - 1];
                for (int32_t j = k - 2; j >= 1; --j)
                    suf[j] = c_mul(yv[j], suf[j + 1]);
                for (int32_t j = 0; j < k; ++j) {
                    ocdd part = j == 0 ? suf[1] : (j == k - 1 ? pre[k - 1] : c_mul(pre[j], suf[j + 1]));
                    ocdd dj = c_scale(c_mul(w, part), (double)expo[b + j]);
                    int64_t at = jbase + (int64_t)pos[b + j] * n_polys + p;
                    store_cdd(J, at, c_add(load_cdd((const double *const *)J, at), dj));
                }
            }
            store_cdd(f, q * n_polys + p, fp);
        }
        free(pre);
        free(suf);
        free(yv);
    }
    if (threads_used)
        *threads_used = used;
    free(pw);
    free(own);
    return 0;
}
