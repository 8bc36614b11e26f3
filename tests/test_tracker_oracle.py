"""Pins of the oracle's path tracker (oracle/tracker.py), on the CPU.

Each test checks the tracker against something other than itself:
  - start solutions: G(x) = 0 and all d_1 ... d_n of them distinct;
  - decoupled squares x_i^2 - c_i: along the homotopy each coordinate obeys
    x_i(t)^2 = ((1-t) gamma + t c_i) / ((1-t) gamma + t), so the end point of
    every path is the continuation of that square root from x_i(0) = +-1,
    followed on a fine grid in t;
  - one variable: the end points are numpy.roots of the polynomial;
  - two quadrics: the x-coordinates of the end points are the roots of the
    Sylvester resultant in x (determinant sampled at five points and
    interpolated), and every end point has a dd residual below 1e-28;
  - a zero leading coefficient (a root at infinity): exactly one of the two
    paths fails and the other ends at the finite root.
"""
import numpy as np
import pytest

import synth
from oracle import ddoracle as O
from oracle import tracker as TR

GAMMA = 0.6 + 0.8j


def _squares(n, seed):
    rng = synth.rng_for(seed)
    c = np.exp(2j * np.pi * rng.uniform(size=n)) * rng.uniform(0.5, 2.0, size=n)
    polys = [[[(i, 2)], []] for i in range(n)]
    coefs = [[1.0, -complex(c[i])] for i in range(n)]
    return synth.system_from_lists(n, polys, coefs), c


def _continued_sqrt(c, x0, gamma=GAMMA, steps=20000):
    """Continue x(t) = sqrt(((1-t) gamma + t c) / ((1-t) gamma + t)) from x0."""
    x = complex(x0)
    for t in np.linspace(0.0, 1.0, steps + 1)[1:]:
        w = np.sqrt(((1 - t) * gamma + t * c) / ((1 - t) * gamma + t))
        x = w if abs(w - x) <= abs(-w - x) else -w
    return x


def test_start_solutions_are_distinct_roots_of_G():
    s = synth.quadric_system(3, 2, 1, seed=11)
    d = TR.total_degrees(s)
    assert list(d) == [2, 2, 2]
    x0 = TR.start_solutions(s, 0, 8)
    assert np.max(np.abs(x0 ** d - 1)) < 1e-14
    dist = np.abs(x0[:, None, :] - x0[None, :, :]).max(axis=2) + 10 * np.eye(8)
    assert dist.min() > 1.9
    # indices wrap modulo the Bezout number
    assert np.array_equal(TR.start_solutions(s, 8, 8), x0)


def test_decoupled_squares_follow_the_closed_form():
    s, c = _squares(3, seed=21)
    x0 = TR.start_solutions(s, 0, 8)
    planes, T, steps, status, res = TR.track(s, x0, gamma=GAMMA)
    assert np.all(status == 0) and np.all(T == 1.0)
    X = planes[0] + 1j * planes[2]
    for p in range(8):
        want = np.array([_continued_sqrt(c[i], x0[p, i]) for i in range(3)])
        assert np.max(np.abs(X[p] - want)) < 1e-8, (p, X[p], want)
    assert np.max(res) < 1e-28
    # the 8 end points are the 8 sign patterns
    assert len({tuple(np.sign(np.round(X[p] / np.sqrt(c), 6).real)) for p in range(8)}) == 8


def test_univariate_end_points_are_numpy_roots():
    rng = synth.rng_for(31)
    coef = np.exp(2j * np.pi * rng.uniform(size=6))  # c_0 .. c_5
    polys = [[[(0, e)] if e else [] for e in range(6)]]
    s = synth.system_from_lists(1, polys, [[complex(v) for v in coef]])
    x0 = TR.start_solutions(s, 0, 5)
    planes, T, steps, status, res = TR.track(s, x0, gamma=GAMMA)
    assert np.all(status == 0)
    got = np.sort_complex((planes[0] + 1j * planes[2])[:, 0])
    want = np.sort_complex(np.roots(coef[::-1]))
    assert np.max(np.abs(got - want)) < 1e-9


def _resultant_roots(s):
    """Roots in x of Res_y(f1, f2) for two quadrics in (x, y) = (x_0, x_1)."""
    def coeffs_in_y(p, x):
        a = np.zeros(3, np.complex128)  # a[e] multiplies y^e
        for m in range(int(s.poly_start[p]), int(s.poly_start[p + 1])):
            c = s.coef[0][m] + 1j * s.coef[2][m]
            ex, ey = 0, 0
            for j in range(int(s.mono_start[m]), int(s.mono_start[m + 1])):
                if s.pos[j] == 0:
                    ex = int(s.exp[j])
                else:
                    ey = int(s.exp[j])
            a[ey] += c * x ** ex
        return a

    def res(x):
        a, b = coeffs_in_y(0, x), coeffs_in_y(1, x)
        S = np.array([[a[2], a[1], a[0], 0], [0, a[2], a[1], a[0]],
                      [b[2], b[1], b[0], 0], [0, b[2], b[1], b[0]]])
        return np.linalg.det(S)

    xs = 1.3 * np.exp(2j * np.pi * np.arange(5) / 5)
    V = np.vander(xs, 5)
    cf = np.linalg.solve(V, np.array([res(x) for x in xs]))
    return np.roots(cf)


def test_two_quadrics_match_the_resultant():
    s = synth.quadric_system(2, 1, 1, seed=41)
    x0 = TR.start_solutions(s, 0, 4)
    planes, T, steps, status, res = TR.track(s, x0, gamma=GAMMA)
    assert np.all(status == 0) and np.max(res) < 1e-28
    X = planes[0] + 1j * planes[2]
    got = np.sort_complex(X[:, 0])
    want = np.sort_complex(_resultant_roots(s))
    assert np.max(np.abs(got - want)) < 1e-7
    # dd residual of the end points, independently of the tracker
    f, _ = O.eval_dd(s, planes, with_jac=False)
    assert np.max(np.hypot(f[0], f[2])) < 1e-28


def test_root_at_infinity_fails_one_path():
    # f = 0 x^2 + x - 1/2: declared degree 2, one finite root 1/2
    s = synth.system_from_lists(1, [[[(0, 2)], [(0, 1)], []]], [[0.0, 1.0, -0.5]])
    x0 = TR.start_solutions(s, 0, 2)
    planes, T, steps, status, res = TR.track(s, x0, gamma=GAMMA, max_steps=400)
    ok = np.nonzero(status == 0)[0]
    assert ok.size == 1 and np.sum(status != 0) == 1
    assert abs(planes[0][ok[0], 0] + planes[1][ok[0], 0] - 0.5) < 1e-28
    assert abs(planes[2][ok[0], 0]) < 1e-28


@pytest.mark.parametrize("n", [3, 4])
def test_quadrics_every_path_reaches_a_distinct_root(n):
    s = synth.quadric_system(n, 2, 2, seed=50 + n)
    P = 2 ** n
    planes, T, steps, status, res = TR.track(s, TR.start_solutions(s, 0, P), gamma=GAMMA)
    assert np.all(status == 0) and np.max(res) < 1e-28
    X = planes[0] + 1j * planes[2]
    dist = np.abs(X[:, None, :] - X[None, :, :]).max(axis=2) + np.eye(P)
    assert dist.min() > 1e-6
