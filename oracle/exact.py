"""ORACLE -- test infrastructure only.

Exact evaluation of a sparse polynomial system and its Jacobian in Gaussian
rationals (pairs of ``fractions.Fraction``), by the definition of Section 2,
equation (1):

    f_p(x)    = sum_{s in p} c_s x^{a_s}
    J[p][i]   = sum_{s in p, i in supp s} c_s a_i x_i^{a_i - 1} prod_{l != i} x_l^{a_l}

A double-double number ``(hi, lo)`` converts exactly as
``Fraction(hi) + Fraction(lo)``.  Meant for tiny systems only.
"""
from __future__ import annotations

from fractions import Fraction as Fr


class GQ:
    """Gaussian rational re + i*im."""

    __slots__ = ("re", "im")

    def __init__(self, re, im=0):
        self.re = Fr(re)
        self.im = Fr(im)

    def __add__(self, o):
        o = _gq(o)
        return GQ(self.re + o.re, self.im + o.im)

    __radd__ = __add__

    def __sub__(self, o):
        o = _gq(o)
        return GQ(self.re - o.re, self.im - o.im)

    def __rsub__(self, o):
        return _gq(o) - self

    def __neg__(self):
        return GQ(-self.re, -self.im)

    def __mul__(self, o):
        o = _gq(o)
        return GQ(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    __rmul__ = __mul__

    def __truediv__(self, o):
        o = _gq(o)
        den = o.re * o.re + o.im * o.im
        num = self * GQ(o.re, -o.im)
        return GQ(num.re / den, num.im / den)

    def __eq__(self, o):
        o = _gq(o)
        return self.re == o.re and self.im == o.im

    def __hash__(self):
        return hash((self.re, self.im))

    def __repr__(self):
        return f"GQ({self.re}, {self.im})"

    def __complex__(self):
        return complex(float(self.re), float(self.im))

    def abs_float(self) -> float:
        return abs(complex(self))


def _gq(v):
    if isinstance(v, GQ):
        return v
    if isinstance(v, complex):
        return GQ(Fr(v.real), Fr(v.imag))
    return GQ(Fr(v), 0)


ZERO = GQ(0, 0)
ONE = GQ(1, 0)
I_UNIT = GQ(0, 1)


def from_dd(re_hi, re_lo, im_hi, im_lo) -> GQ:
    return GQ(Fr(float(re_hi)) + Fr(float(re_lo)), Fr(float(im_hi)) + Fr(float(im_lo)))


def power(x: GQ, e: int) -> GQ:
    r = ONE
    for _ in range(e):
        r = r * x
    return r


def coefficients(system):
    c = system.coef
    return [from_dd(c[0][s], c[1][s], c[2][s], c[3][s]) for s in range(system.n_monos)]


def point_from_planes(planes, row: int = 0):
    n = planes[0].shape[-1]
    pl = [a.reshape(-1, n)[row] for a in planes]
    return [from_dd(pl[0][i], pl[1][i], pl[2][i], pl[3][i]) for i in range(n)]


def eval_exact(system, x, coefs=None, with_jac: bool = True):
    """Exact f (list over polynomials) and J (J[p][i], list of lists) at the
    Gaussian-rational point ``x`` (list of GQ)."""
    coefs = coefficients(system) if coefs is None else coefs
    n, npoly = system.n_vars, system.n_polys
    f = [ZERO] * npoly
    J = [[ZERO] * n for _ in range(npoly)] if with_jac else None
    for p in range(npoly):
        fp = ZERO
        for s in range(int(system.poly_start[p]), int(system.poly_start[p + 1])):
            pos, ex = system.monomial(s)
            c = coefs[s]
            v = c
            for i, e in zip(pos, ex):
                v = v * power(x[int(i)], int(e))
            fp = fp + v
            if with_jac:
                for j, (i, e) in enumerate(zip(pos, ex)):
                    d = c * int(e) * power(x[int(i)], int(e) - 1)
                    for l, (i2, e2) in enumerate(zip(pos, ex)):
                        if l != j:
                            d = d * power(x[int(i2)], int(e2))
                    J[p][int(i)] = J[p][int(i)] + d
        f[p] = fp
    return f, J


def lagrange_derivative_at_zero(values, nodes):
    """Exact derivative at t = 0 of the interpolating polynomial through
    ``(nodes[j], values[j])`` (Gaussian rationals, distinct rational nodes)."""
    total = ZERO
    m = len(nodes)
    for j in range(m):
        # L_j'(0) = sum_{r != j} 1/(t_j - t_r) * prod_{l != j, r} (0 - t_l)/(t_j - t_l)
        dj = Fr(0)
        for r in range(m):
            if r == j:
                continue
            term = Fr(1) / (nodes[j] - nodes[r])
            for l in range(m):
                if l != j and l != r:
                    term *= (Fr(0) - nodes[l]) / (nodes[j] - nodes[l])
            dj += term
        total = total + values[j] * GQ(dj, 0)
    return total
