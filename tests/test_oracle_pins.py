"""Pins for the oracle (CPU only).

The oracle is the definition of Section 2, equation (1).  These tests tie it
to facts that do not come from the oracle itself:

* the paper's worked common-factor example (Section 3.1, golden file);
* closed forms and special cases that reduce to textbook or library results
  (the Speelpenning product, linear systems against numpy's matmul);
* identities that hold exactly for polynomials: Euler's identity on
  homogeneous systems, and the derivative recovered exactly from values of
  ``f`` alone by polynomial interpolation along a coordinate;
* the exactness of the error-free transformations and the published error
  bounds of the double-word operations, checked in rational arithmetic;
* agreement of the dd evaluator with the exact-rational evaluator on small
  systems (brute force), and invariance under relabelling.
"""
import math
import os
import random
from fractions import Fraction as Fr

import numpy as np
import pytest

import synth
from oracle import ddoracle as O
from oracle import exact as E

U = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _fr_dd(h, l):
    return Fr(float(h)) + Fr(float(l))


def _gq_planes(planes, idx):
    return E.from_dd(planes[0][idx], planes[1][idx], planes[2][idx], planes[3][idx])


def _dyadic_point(n, seed, bits=40):
    """Unit-circle-ish point whose coordinates are multiples of 2^-bits (lo = 0),
    so that shifting a coordinate by small dyadic steps stays exact."""
    rng = synth.rng_for(seed)
    th = rng.uniform(0, 2 * math.pi, n)
    s = 2.0 ** bits
    re = np.round(np.cos(th) * s) / s
    im = np.round(np.sin(th) * s) / s
    z = np.zeros(n)
    return (re.reshape(1, n), z.reshape(1, n), im.reshape(1, n), z.reshape(1, n))


# ---------------------------------------------------------------------------
# exact evaluator: pins against the paper and the mathematics
# ---------------------------------------------------------------------------

def _read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split(":")
            out[k.strip()] = [int(t) for t in v.split()]
    return out


def test_exact_common_factor_worked_example():
    """Section 3.1: every partial of x1^3 x2^7 x3^2 equals a_j times the
    common factor x1^2 x2^6 x3 times the partial of x1 x2 x3."""
    g = _read_golden("common_factor_example.txt")
    a, cf_e = g["monomial_exponents"], g["common_factor_exponents"]
    assert cf_e == [e - 1 for e in a]
    sys = synth.system_from_lists(3, [[[(0, a[0]), (1, a[1]), (2, a[2])]]], [[1.0]])
    x = [E.GQ(Fr(3, 4), Fr(1, 8)), E.GQ(Fr(-5, 16), Fr(1, 2)), E.GQ(Fr(7, 8), Fr(-3, 32))]
    f, J = E.eval_exact(sys, x)
    cf = E.power(x[0], cf_e[0]) * E.power(x[1], cf_e[1]) * E.power(x[2], cf_e[2])
    speel = [x[1] * x[2], x[0] * x[2], x[0] * x[1]]
    for j in range(3):
        assert J[0][j] == cf * speel[j] * a[j]
    assert f[0] == cf * x[0] * x[1] * x[2]


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_exact_speelpenning_partials_by_quotient(k):
    """Speelpenning's product x_1...x_k: each partial times its own variable
    gives back the product (x_i * d/dx_i is the identity on a multilinear
    monomial)."""
    sys = synth.system_from_lists(k, [[[(i, 1) for i in range(k)]]], [[1.0]])
    rng = random.Random(k)
    x = [E.GQ(Fr(rng.randint(1, 63), 32), Fr(rng.randint(-63, 63), 64)) for _ in range(k)]
    f, J = E.eval_exact(sys, x)
    for i in range(k):
        assert J[0][i] == f[0] / x[i]


def test_exact_linear_system_matches_numpy_matmul():
    """A linear system f = A x + b (k = 1, exponent 1, plus constants):
    f agrees with numpy's matrix product and J equals A."""
    rng = np.random.default_rng(5)
    n = 6
    A = rng.integers(-8, 9, (n, n)) + 1j * rng.integers(-8, 9, (n, n))
    b = rng.integers(-8, 9, n) + 1j * rng.integers(-8, 9, n)
    x = (rng.integers(-16, 17, n) + 1j * rng.integers(-16, 17, n)) / 8.0
    polys, coefs = [], []
    for p in range(n):
        polys.append([[(i, 1)] for i in range(n)] + [[]])
        coefs.append([complex(A[p, i]) for i in range(n)] + [complex(b[p])])
    sys = synth.system_from_lists(n, polys, coefs)
    xg = [E.GQ(Fr(v.real), Fr(v.imag)) for v in x]
    f, J = E.eval_exact(sys, xg)
    ref = A @ x + b      # exact in float64: small dyadic integers
    for p in range(n):
        assert complex(f[p]) == ref[p]
        for i in range(n):
            assert J[p][i] == E.GQ(Fr(A[p, i].real), Fr(A[p, i].imag))


def test_exact_euler_identity_homogeneous():
    """Euler: sum_i x_i df/dx_i = D f for f homogeneous of degree D."""
    D = 7
    sys = synth.homogeneous_system(6, 5, 3, D, seed=11)
    pts = _dyadic_point(6, 12, bits=12)
    x = E.point_from_planes(pts)
    f, J = E.eval_exact(sys, x)
    for p in range(sys.n_polys):
        lhs = E.ZERO
        for i in range(6):
            lhs = lhs + x[i] * J[p][i]
        assert lhs == f[p] * D


def test_exact_derivative_from_values_by_interpolation():
    """J[p][i] equals the exact derivative at t=0 of t -> f_p(x + t e_i),
    recovered from values of f alone by interpolation (exact because the
    restriction is a polynomial of degree <= max exponent)."""
    sys = synth.regular_system(5, 4, 3, (1, 4), seed=3)
    pts = _dyadic_point(5, 4, bits=10)
    x = E.point_from_planes(pts)
    f, J = E.eval_exact(sys, x)
    coefs = E.coefficients(sys)
    deg = sys.max_exp
    nodes = [Fr(j - deg // 2, 4) for j in range(deg + 2)]
    for i in range(5):
        vals = []
        for t in nodes:
            xt = list(x)
            xt[i] = x[i] + E.GQ(t, 0)
            vals.append(E.eval_exact(sys, xt, coefs, with_jac=False)[0])
        for p in range(sys.n_polys):
            d = E.lagrange_derivative_at_zero([v[p] for v in vals], nodes)
            assert d == J[p][i]


def test_exact_structural_zeros():
    """J[p][i] is exactly zero when no monomial of f_p contains x_i."""
    sys = synth.regular_system(9, 2, 2, (1, 3), seed=8)
    x = E.point_from_planes(synth.points(1, 9, 9))
    f, J = E.eval_exact(sys, x)
    for p in range(sys.n_polys):
        used = set()
        for s in range(int(sys.poly_start[p]), int(sys.poly_start[p + 1])):
            used.update(int(v) for v in sys.monomial(s)[0])
        for i in range(9):
            if i not in used:
                assert J[p][i] == E.ZERO


# ---------------------------------------------------------------------------
# dd primitives: exactness and published error bounds, in rationals
# ---------------------------------------------------------------------------

def _adversarial_doubles(seed, n=400):
    rng = np.random.default_rng(seed)
    vals = list(rng.standard_normal(n) * 2.0 ** rng.integers(-60, 60, n))
    vals += [1.0, -1.0, 0.0, -0.0, 1.0 + 2 ** -52, 1.0 - 2 ** -53, 2 ** 500, -2 ** -500,
             3.0 * 2 ** -1074, 1e-300, 1 - 1e-16, 0.1, 1 / 3]
    return [float(v) for v in vals]


def test_two_sum_and_two_prod_are_error_free():
    v = _adversarial_doubles(1)
    rng = random.Random(2)
    for _ in range(3000):
        a, b = rng.choice(v), rng.choice(v)
        s, e = O.two_sum(a, b)
        assert Fr(s) + Fr(e) == Fr(a) + Fr(b)
        assert s == a + b
        if abs(a) < 2 ** 900 and abs(b) < 2 ** 900 and abs(a * b) > 2 ** -960:
            p, e = O.two_prod(a, b)
            assert Fr(p) + Fr(e) == Fr(a) * Fr(b)
            assert p == a * b


def _rand_dd(rng):
    h = float(rng.standard_normal() * 2.0 ** rng.integers(-20, 20))
    # low words on different binary grids, so that sums of low words round
    l = float(rng.uniform(-0.5, 0.5) * np.spacing(abs(h)) * 2.0 ** -int(rng.integers(0, 12)))
    return (h, l)


def test_dd_add_mul_div_error_bounds():
    """Accurate double-word sum: relative error <= 3u^2/(1-4u); double-word
    product without FMA: <= 7u^2 (Joldes, Muller, Popescu 2017); division
    by long division: checked at <= 16u^2.  Outputs are normalized."""
    rng = np.random.default_rng(7)
    worst = {"add": 0.0, "mul": 0.0, "div": 0.0}
    for t in range(4000):
        x, y = _rand_dd(rng), _rand_dd(rng)
        if t % 5 == 0:  # cancellation
            y = (-x[0] * (1 + 2 ** -40),
                 float(rng.uniform(-0.5, 0.5) * np.spacing(abs(x[0])) * 2.0 ** -int(rng.integers(0, 12))))
        X, Y = _fr_dd(*x), _fr_dd(*y)
        for name, fn, exact in (("add", O.dd_add, X + Y), ("mul", O.dd_mul, X * Y),
                                ("div", O.dd_div, X / Y if Y != 0 else None)):
            if exact is None:
                continue
            zh, zl = fn(x, y)
            assert abs(zl) <= 0.5 * np.spacing(abs(zh)) or zh == 0.0
            if exact != 0:
                rel = abs((Fr(zh) + Fr(zl) - exact) / exact)
                worst[name] = max(worst[name], float(rel))
    assert worst["add"] <= 3 * U * U / (1 - 4 * U)
    assert worst["mul"] <= 7 * U * U
    assert worst["div"] <= 16 * U * U


# ---------------------------------------------------------------------------
# dd and FP64 evaluators against the exact evaluator (brute force, tiny)
# ---------------------------------------------------------------------------

def _special_system():
    """Hand-made system covering k = 0, 1, 2, high exponents, a zero
    coefficient and a duplicated monomial."""
    polys = [
        [[], [(0, 1)], [(1, 2), (3, 1)], [(0, 5), (2, 8)]],
        [[(0, 1), (1, 1), (2, 1), (3, 1)], [(0, 1), (1, 1), (2, 1), (3, 1)], [(2, 3)]],
        [[(1, 1), (2, 2)], [(3, 6)], []],
        [[(0, 2), (1, 3), (2, 1), (3, 2)]],
    ]
    rng = synth.rng_for(77)
    coefs = []
    for monos in polys:
        pl = synth.unit_circle_dd(rng, (len(monos),))
        coefs.append([tuple(float(a[j]) for a in pl) for j in range(len(monos))])
    coefs[0][1] = (0.0, 0.0, 0.0, 0.0)
    return synth.system_from_lists(4, polys, coefs)


def _max_scaled_err_vs_exact(sys, pts, npts):
    f, J = O.eval_dd(sys, pts)
    Sf, SJ = O.scales(sys, pts[0], pts[2])
    coefs = E.coefficients(sys)
    worst = 0.0
    n, npoly = sys.n_vars, sys.n_polys
    for q in range(npts):
        x = E.point_from_planes(pts, q)
        fe, Je = E.eval_exact(sys, x, coefs)
        for p in range(npoly):
            err = (_gq_planes(f, (q, p)) - fe[p]).abs_float()
            worst = max(worst, err / Sf[q, p])
            for i in range(n):
                got = _gq_planes(J, (q, i, p))
                if SJ[q, i, p] == 0.0:
                    assert got == E.ZERO and Je[p][i] == E.ZERO
                else:
                    worst = max(worst, (got - Je[p][i]).abs_float() / SJ[q, i, p])
    return worst


def test_dd_oracle_matches_exact_on_tiny_workload():
    sys, pts = synth.tiny_workload()
    assert _max_scaled_err_vs_exact(sys, pts, 1) < 1e-30


def test_dd_oracle_matches_exact_on_special_cases():
    sys = _special_system()
    pts = synth.points(3, 4, 99)
    assert _max_scaled_err_vs_exact(sys, pts, 3) < 1e-30


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_dd_oracle_matches_exact_random_small(seed):
    sys = synth.regular_system(7, 5, 3, (1, 4), seed=seed)
    pts = synth.points(2, 7, seed + 100)
    assert _max_scaled_err_vs_exact(sys, pts, 2) < 1e-30


def test_f64_oracle_matches_exact():
    sys, pts = synth.tiny_workload()
    (fr, fi), (Jr, Ji) = O.eval_f64(sys, pts[0], pts[2])
    Sf, SJ = O.scales(sys, pts[0], pts[2])
    # the FP64 evaluator sees the points and coefficients rounded to FP64
    sys64 = synth.System(sys.n_vars, sys.n_polys, sys.poly_start, sys.mono_start, sys.pos,
                         sys.exp, (sys.coef[0], 0 * sys.coef[1], sys.coef[2], 0 * sys.coef[3]))
    x = [E.GQ(Fr(pts[0][0, i]), Fr(pts[2][0, i])) for i in range(8)]
    fe, Je = E.eval_exact(sys64, x)
    worst = 0.0
    for p in range(8):
        worst = max(worst, abs(complex(fr[0, p], fi[0, p]) - complex(fe[p])) / Sf[0, p])
        for i in range(8):
            if SJ[0, i, p] > 0:
                worst = max(worst, abs(complex(Jr[0, i, p], Ji[0, i, p]) - complex(Je[p][i])) / SJ[0, i, p])
    assert worst < 1e-14


# ---------------------------------------------------------------------------
# dd evaluator on larger systems: identities that hold for any polynomial
# ---------------------------------------------------------------------------

def test_dd_oracle_euler_identity_medium():
    D = 12
    n = 24
    sys = synth.homogeneous_system(n, 24, 6, D, seed=21)
    pts = synth.points(2, n, 22)
    f, J = O.eval_dd(sys, pts)
    Sf, _ = O.scales(sys, pts[0], pts[2], with_jac=False)
    for q in range(2):
        x = E.point_from_planes(pts, q)
        for p in range(n):
            lhs = E.ZERO
            for i in range(n):
                lhs = lhs + x[i] * _gq_planes(J, (q, i, p))
            r = (lhs - _gq_planes(f, (q, p)) * D).abs_float()
            assert r <= 1e-29 * 2 * D * Sf[q, p]


def test_dd_oracle_derivative_identity_medium():
    """J from the dd evaluator against the derivative recovered exactly from
    dd values of f at shifted points (interpolation weights in rationals)."""
    n = 16
    sys = synth.regular_system(n, 32, 6, (1, 4), seed=31)
    pts = _dyadic_point(n, 32, bits=40)
    f, J = O.eval_dd(sys, pts)
    _, SJ = O.scales(sys, pts[0], pts[2])
    deg = sys.max_exp
    nodes = [Fr(j - deg // 2, 4) for j in range(deg + 1)]
    for i in range(0, n, 3):
        vals, scl = [], []
        for t in nodes:
            sh = [a.copy() for a in pts]
            sh[0][0, i] = float(Fr(pts[0][0, i]) + t)   # exact: few significant bits
            assert Fr(sh[0][0, i]) == Fr(pts[0][0, i]) + t
            fv, _ = O.eval_dd(sys, sh, with_jac=False)
            sf, _ = O.scales(sys, sh[0], sh[2], with_jac=False)
            vals.append(fv)
            scl.append(sf)
        weights_mag = []
        for j in range(len(nodes)):
            basis = [E.ZERO] * len(nodes)
            basis[j] = E.ONE
            weights_mag.append(abs(float(E.lagrange_derivative_at_zero(basis, nodes).re)))
        for p in range(n):
            d = E.lagrange_derivative_at_zero([_gq_planes(v, (0, p)) for v in vals], nodes)
            got = _gq_planes(J, (0, i, p))
            bound = 1e-29 * (sum(w * s[0, p] for w, s in zip(weights_mag, scl)) + SJ[0, i, p])
            assert (got - d).abs_float() <= bound


def test_dd_oracle_relabelling_invariance():
    """Shuffling monomials and renaming variables permutes the outputs."""
    n = 12
    sys = synth.regular_system(n, 20, 4, (1, 3), seed=41)
    pts = synth.points(1, n, 42)
    rng = np.random.default_rng(43)
    sigma = rng.permutation(n)              # old var i -> new var sigma[i]
    polys, coefs = [], []
    for p in range(n):
        order = rng.permutation(np.arange(int(sys.poly_start[p]), int(sys.poly_start[p + 1])))
        monos, cs = [], []
        for s in order:
            pos, ex = sys.monomial(int(s))
            mono = sorted((int(sigma[v]), int(e)) for v, e in zip(pos, ex))
            monos.append(mono)
            cs.append(tuple(float(a[s]) for a in sys.coef))
        polys.append(monos)
        coefs.append(cs)
    sys2 = synth.system_from_lists(n, polys, coefs)
    pts2 = tuple(np.empty_like(a) for a in pts)
    for a, b in zip(pts, pts2):
        b[0, sigma] = a[0, :]
    f, J = O.eval_dd(sys, pts)
    f2, J2 = O.eval_dd(sys2, pts2)
    Sf, SJ = O.scales(sys, pts[0], pts[2])
    assert np.all(O.dd_diff_abs(f, f2) <= 1e-30 * Sf)
    Jp = tuple(a[:, sigma, :] for a in J2)
    assert np.all(O.dd_diff_abs(J, Jp) <= 1e-30 * SJ + 0.0)


def test_f64_oracle_central_differences():
    """Coarse sanity check: FP64 Jacobian against central differences of f."""
    n = 10
    sys = synth.regular_system(n, 12, 3, (1, 3), seed=51)
    pts = synth.points(1, n, 52)
    (fr, fi), (Jr, Ji) = O.eval_f64(sys, pts[0], pts[2])
    h = 1e-5
    for i in range(n):
        xp, xm = pts[0].copy(), pts[0].copy()
        xp[0, i] += h
        xm[0, i] -= h
        (a, b), _ = O.eval_f64(sys, xp, pts[2], with_jac=False)
        (c, d), _ = O.eval_f64(sys, xm, pts[2], with_jac=False)
        fd = ((a - c) + 1j * (b - d)) / (2 * h)
        got = Jr[0, i] + 1j * Ji[0, i]
        assert np.all(np.abs(fd[0] - got) <= 1e-7 * (1 + np.abs(got)))


# ---------------------------------------------------------------------------
# dd linear solve and plain dd Newton
# ---------------------------------------------------------------------------

def test_dd_solve_recovers_exact_solution():
    n = 9
    rng = synth.rng_for(61)
    A = synth.unit_circle_dd(rng, (n, n))       # A[r][c] stored column-major below
    xt = [E.GQ(Fr(int(v), 64), Fr(int(w), 128)) for v, w in zip(rng.integers(-64, 64, n), rng.integers(-128, 128, n))]
    Ag = [[E.from_dd(A[0][r, c], A[1][r, c], A[2][r, c], A[3][r, c]) for c in range(n)] for r in range(n)]
    b = []
    for r in range(n):
        acc = E.ZERO
        for c in range(n):
            acc = acc + Ag[r][c] * xt[c]
        b.append(acc)
    # b rounded to dd (exact rational -> hi, lo)
    bpl = [np.zeros(n) for _ in range(4)]
    for r in range(n):
        for comp, (hi_i, lo_i) in ((b[r].re, (0, 1)), (b[r].im, (2, 3))):
            hi = float(comp)
            bpl[hi_i][r] = hi
            bpl[lo_i][r] = float(comp - Fr(hi))
    Acol = [a.T.reshape(-1) for a in A]         # column-major
    st, x = O.solve_dd(Acol, bpl)
    assert st == 0
    for c in range(n):
        assert (E.from_dd(x[0][c], x[1][c], x[2][c], x[3][c]) - xt[c]).abs_float() < 1e-27


@pytest.mark.parametrize("seed", [0, 1])
def test_dd_newton_converges_to_known_root(seed):
    n = 8
    sys, xstar = synth.known_root_system(n, 6, 3, (1, 3), seed=500 + seed)
    # exact check of the construction: f(x*) is within dd rounding of zero
    xs = [E.from_dd(xstar[0][i], xstar[1][i], xstar[2][i], xstar[3][i]) for i in range(n)]
    f0, _ = E.eval_exact(sys, xs, with_jac=False)
    assert max(v.abs_float() for v in f0) < 1e-31
    starts = synth.perturbed_starts(xstar, 3, 1e-6, seed=600 + seed)
    x, res, iters, status = O.newton_dd(sys, starts, tol=1e-28, max_iter=8)
    assert np.all(status == 0)
    assert np.all(res < 1e-28)
    assert np.all(iters <= 5)
    coefs = E.coefficients(sys)
    for q in range(3):
        xq = [E.from_dd(x[0][q, i], x[1][q, i], x[2][q, i], x[3][q, i]) for i in range(n)]
        fq, _ = E.eval_exact(sys, xq, coefs, with_jac=False)
        assert max(v.abs_float() for v in fq) < 1e-28
        assert max((a - b).abs_float() for a, b in zip(xq, xs)) < 1e-26


@pytest.mark.parametrize("shape", [(8, 6, 3, (1, 3)), (5, 40, 4, (1, 5))])
def test_known_root_on_a_coefficient_grid_is_exact(shape):
    """With coefficients on a 2^-40 grid the constant term makes x* an exact
    root: f(x*) = 0 in Gaussian rationals (the quad-double Newton tests rely
    on it)."""
    n, m, k, ex = shape
    sys, xstar = synth.known_root_system(n, m, k, ex, seed=520 + n, coef_grid=40)
    assert all(np.all(sys.coef[q] == 0.0) for q in (1, 3))
    xs = [E.from_dd(xstar[0][i], xstar[1][i], xstar[2][i], xstar[3][i]) for i in range(n)]
    f0, _ = E.eval_exact(sys, xs, with_jac=False)
    assert all(v.re == 0 and v.im == 0 for v in f0)
    # and the grid is what makes it exact: without it the rounding shows
    sys2, _ = synth.known_root_system(n, m, k, ex, seed=520 + n)
    f2, _ = E.eval_exact(sys2, xs, with_jac=False)
    assert any(v.re != 0 or v.im != 0 for v in f2)


def test_dd_newton_reports_singular_and_nonconvergence():
    n = 4
    # duplicated polynomial -> singular Jacobian everywhere
    polys = [[[(0, 1), (1, 1)], [(2, 2)], []]] * 2 + [[[(2, 1)], [(3, 1)], []], [[(3, 2)], [(0, 1)], []]]
    coefs = [[1.0, 0.5, -0.25]] * 2 + [[1.0, -1.0, 0.5], [1.0, 2.0, -1.0]]
    sys = synth.system_from_lists(n, polys, coefs)
    st0 = tuple(np.full((1, n), v) for v in (0.3, 0.0, 0.2, 0.0))
    _, _, _, status = O.newton_dd(sys, st0, tol=1e-28, max_iter=5)
    assert status[0] == 2
    # a regular system stopped after 0 iterations is not converged
    sys2, xstar = synth.known_root_system(6, 4, 2, (1, 2), seed=3)
    starts = synth.perturbed_starts(xstar, 1, 1e-3, seed=4)
    _, _, iters, status = O.newton_dd(sys2, starts, tol=1e-28, max_iter=0)
    assert status[0] == 1 and iters[0] == 0
    bad = tuple(a.copy() for a in starts)
    bad[0][0, 0] = np.nan
    _, _, _, status = O.newton_dd(sys2, bad, tol=1e-28, max_iter=3)
    assert status[0] == 3


# ---------------------------------------------------------------------------
# magnitude scales of the error metric (orc_scales)
#
# S(f_p) = sum_s |c_s| |x^{a_s}| and S(J[p][i]) = sum_{s: i in supp s}
# |c_s| a_i |x_i|^{a_i - 1} prod_{l != i} |x_l|^{a_l}.  Because the modulus is
# multiplicative, these are exactly the value and the partial derivatives of
# the "magnitude system" (same supports, coefficients |c_s|) at the real
# point |x|; the exact-rational evaluator, pinned above, computes those.
# ---------------------------------------------------------------------------

_TRIPLES = [(3, 4, 5), (5, 12, 13), (8, 15, 17), (7, 24, 25), (20, 21, 29), (12, 35, 37)]
_RADII = [Fr(1, 2), Fr(5, 8), Fr(3, 4), Fr(7, 8), Fr(1), Fr(5, 4), Fr(3, 2), Fr(7, 4), Fr(2)]


def _pythagorean(rng, radius):
    """(radius * (a + i b) / c as two doubles, exact modulus radius) for a
    random Pythagorean triple (a, b, c), with random signs and order."""
    a, b, c = _TRIPLES[int(rng.integers(len(_TRIPLES)))]
    if rng.integers(2):
        a, b = b, a
    sa, sb = (1 if rng.integers(2) else -1), (1 if rng.integers(2) else -1)
    return float(radius * sa * a / c), float(radius * sb * b / c)


def _non_unit_system(n, m, k, exp_range, seed, homogeneous_degree=None):
    """A random system whose coefficients and point have exact dyadic moduli
    in [1/2, 2] (Pythagorean directions), exponents >= 2 included.  Returns
    the system, the point planes, the exact moduli |c_s| and |x_i|."""
    if homogeneous_degree is None:
        base = synth.regular_system(n, m, k, exp_range, seed=seed)
    else:
        base = synth.homogeneous_system(n, m, k, homogeneous_degree, seed=seed)
    rng = np.random.default_rng(seed + 1)
    M = base.n_monos
    cmag = [_RADII[int(rng.integers(len(_RADII)))] for _ in range(M)]
    cre, cim = zip(*[_pythagorean(rng, r) for r in cmag])
    z = np.zeros(M)
    sys = synth.System(base.n_vars, base.n_polys, base.poly_start, base.mono_start, base.pos,
                       base.exp, (np.array(cre), z, np.array(cim), z.copy()))
    xmag = [_RADII[int(rng.integers(len(_RADII)))] for _ in range(n)]
    xre, xim = zip(*[_pythagorean(rng, r) for r in xmag])
    zx = np.zeros((1, n))
    pts = (np.array(xre).reshape(1, n), zx, np.array(xim).reshape(1, n), zx.copy())
    return sys, pts, cmag, xmag


def _magnitude_system(sys, cmag):
    M = sys.n_monos
    re = np.array([float(c) for c in cmag])
    z = np.zeros(M)
    return synth.System(sys.n_vars, sys.n_polys, sys.poly_start, sys.mono_start, sys.pos,
                        sys.exp, (re, z, z.copy(), z.copy()))


@pytest.mark.parametrize("seed", [71, 72])
def test_scales_are_the_magnitude_system_at_the_modulus_point(seed):
    """orc_scales against the exact value and Jacobian of the magnitude
    system (coefficients |c_s|) at |x|, at points of modulus 1/2 .. 2 and
    exponents up to 4.  The doubles of the Pythagorean directions are
    rounded, so |x_i| and |c_s| as the oracle sees them differ from the
    exact radii by a few ulps: the bar is 1e-12 relative."""
    sys, pts, cmag, xmag = _non_unit_system(6, 7, 3, (1, 4), seed)
    Sf, SJ = O.scales(sys, pts[0], pts[2])
    fe, Je = E.eval_exact(_magnitude_system(sys, cmag), [E.GQ(r, 0) for r in xmag])
    for p in range(sys.n_polys):
        assert fe[p].im == 0 and fe[p].re > 0
        assert abs(Sf[0, p] - float(fe[p].re)) <= 1e-12 * float(fe[p].re)
        for i in range(sys.n_vars):
            ref = float(Je[p][i].re)
            if ref == 0.0:
                assert SJ[0, i, p] == 0.0
            else:
                assert abs(SJ[0, i, p] - ref) <= 1e-12 * ref


def test_scales_euler_identity_homogeneous():
    """The magnitude system of a homogeneous system is homogeneous of the
    same degree D, so sum_i |x_i| S(J[p][i]) = D S(f_p), at a point with
    moduli 1/2 .. 2."""
    D = 9
    sys, pts, cmag, xmag = _non_unit_system(8, 6, 4, None, 73, homogeneous_degree=D)
    Sf, SJ = O.scales(sys, pts[0], pts[2])
    ax = np.hypot(pts[0][0], pts[2][0])
    for p in range(sys.n_polys):
        lhs = float(np.sum(ax * SJ[0, :, p]))
        assert abs(lhs - D * Sf[0, p]) <= 1e-13 * D * Sf[0, p]


def test_scales_equal_the_values_for_positive_data():
    """With positive real coefficients and a positive real point every term
    is a positive real, so the sums of magnitudes are the values and
    derivatives themselves (the triangle inequality with equality):
    S(f_p) = f_p and S(J[p][i]) = J[p][i], against the exact evaluator."""
    base = synth.regular_system(7, 6, 3, (1, 4), seed=74)
    rng = np.random.default_rng(75)
    M = base.n_monos
    c = np.array([float(_RADII[int(rng.integers(len(_RADII)))]) for _ in range(M)])
    z = np.zeros(M)
    sys = synth.System(base.n_vars, base.n_polys, base.poly_start, base.mono_start, base.pos,
                       base.exp, (c, z, z.copy(), z.copy()))
    xv = [_RADII[int(rng.integers(len(_RADII)))] for _ in range(7)]
    xr = np.array([[float(v) for v in xv]])
    Sf, SJ = O.scales(sys, xr, np.zeros_like(xr))
    fe, Je = E.eval_exact(sys, [E.GQ(v, 0) for v in xv])
    for p in range(sys.n_polys):
        assert abs(Sf[0, p] - float(fe[p].re)) <= 1e-14 * float(fe[p].re)
        for i in range(7):
            ref = float(Je[p][i].re)
            assert abs(SJ[0, i, p] - ref) <= 1e-14 * ref


def test_scales_on_the_unit_circle():
    """Special case |x_i| = 1: S(f_p) = sum_s |c_s| and S(J[p][i]) =
    sum over the monomials of f_p containing x_i of a_i |c_s|."""
    sys, pts = synth.tiny_workload()
    Sf, SJ = O.scales(sys, pts[0], pts[2])
    cabs = np.hypot(sys.coef[0], sys.coef[2])
    for p in range(sys.n_polys):
        s0, s1 = int(sys.poly_start[p]), int(sys.poly_start[p + 1])
        assert abs(Sf[0, p] - cabs[s0:s1].sum()) <= 1e-14 * Sf[0, p]
        ref = np.zeros(sys.n_vars)
        for s in range(s0, s1):
            for v, e in zip(*sys.monomial(s)):
                ref[int(v)] += e * cabs[s]
        assert np.allclose(SJ[0, :, p], ref, rtol=1e-14, atol=0.0)


# ---------------------------------------------------------------------------
# fast mode (CPU throughput baseline) against the definitional evaluator
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(8, 8, 4, (1, 2)), (20, 30, 7, (1, 5)), (40, 16, 1, (1, 3)),
                                   (12, 10, 2, (1, 3))])
def test_fast_mode_matches_definitional_evaluator(shape):
    """Within 1e-30 of the term-magnitude scale at every output (the two
    round products in different orders), exact zeros where x_i does not
    occur, and the same bits for 1 and 3 threads."""
    n, m, k, er = shape
    sys = synth.regular_system(n, m, k, er, seed=81 + n)
    pts = synth.points(3, n, 82 + n)
    f, J = O.eval_dd(sys, pts)
    ff, Jf, used = O.eval_dd_fast(sys, pts, threads=3)
    ff1, Jf1, used1 = O.eval_dd_fast(sys, pts, threads=1)
    assert used1 == 1
    Sf, SJ = O.scales(sys, pts[0], pts[2])
    assert np.all(O.dd_diff_abs(f, ff) <= 1e-30 * Sf)
    pos = SJ > 0
    assert np.all(O.dd_diff_abs(J, Jf)[pos] <= 1e-30 * SJ[pos])
    for a in Jf:
        assert np.all(a[~pos] == 0.0)
    for a, b in zip(ff + Jf, ff1 + Jf1):
        assert np.array_equal(a, b)


def test_fast_mode_special_cases_and_selection():
    """Constants, k = 1 and 2, a zero coefficient, a repeated monomial and
    high exponents; then a selection of polynomials."""
    sys = _special_system()
    pts = synth.points(2, 4, 83)
    f, J = O.eval_dd(sys, pts)
    ff, Jf, _ = O.eval_dd_fast(sys, pts)
    Sf, SJ = O.scales(sys, pts[0], pts[2])
    assert np.all(O.dd_diff_abs(f, ff) <= 1e-30 * Sf)
    pos = SJ > 0
    assert np.all(O.dd_diff_abs(J, Jf)[pos] <= 1e-30 * SJ[pos])
    fs, Js, _ = O.eval_dd_fast(sys, pts, polys=[1, 3])
    for a, b in zip(fs, ff):
        assert np.array_equal(a[:, [1, 3]], b[:, [1, 3]]) and np.all(np.isnan(a[:, [0, 2]]))
