"""Known-root systems at a generic point (test infrastructure).

A regular random system gets one constant monomial per polynomial, last,
with c_0 = -sum_s c_s x*^{a_s}, so that the point x* is a root.  Here x* is
a generic unit-circle double-double point (not a root of unity), so the
monomial values at x* are not exact units and Newton's convergence is
measured away from exact products.

The sum is formed exactly enough in fixed point: double-double inputs are
taken as integer multiples of 2^-SCALE (SCALE = 192 bits; exact unless a
word is below 2^-139, else truncated by less than 2^-192), products are
truncated to that grid (error below 2^-186 per product for factors of
modulus up to 2), and the constant is rounded once to double-double.  The remaining error of f(x*) is that one
rounding, at most u^2 |c_0| with u = 2^-53.  Vectorized over monomials with
numpy object arrays of Python integers.
"""
from __future__ import annotations

import math

import numpy as np

import synth

SCALE = 192


def _fixed(v: np.ndarray) -> np.ndarray:
    """Doubles -> exact integers at scale 2^SCALE (object array)."""
    out = np.empty(v.shape, dtype=object)
    flat, of = v.reshape(-1), out.reshape(-1)
    for t in range(flat.size):
        m, e = math.frexp(float(flat[t]))
        mant = int(m * (1 << 53))
        sh = e - 53 + SCALE
        of[t] = mant << sh if sh >= 0 else -((-mant) >> -sh) if mant < 0 else mant >> -sh
    return out


def _to_dd(v: int):
    """An integer at scale 2^SCALE rounded to double-double (hi, lo)."""
    hi = math.ldexp(float(v), -SCALE) if v else 0.0
    num, den = hi.as_integer_ratio()
    rem = v - num * ((1 << SCALE) // den)
    lo = math.ldexp(float(rem), -SCALE) if rem else 0.0
    return hi, lo


def known_root_system_generic(n: int, m: int, k: int, exp_range=(1, 3), seed: int = 0):
    """``(system, xstar_planes)``: a regular system of n polynomials with m
    monomials (k variables, exponents in exp_range) plus a constant last in
    each polynomial, vanishing at a random unit-circle dd point x*."""
    base = synth.regular_system(n, m, k, exp_range, seed)
    xs = synth.points(1, n, seed + 4241)
    xstar = tuple(a[0].copy() for a in xs)
    M = base.n_monos
    d = int(base.exp.max())
    xr = _fixed(xstar[0]) + _fixed(xstar[1])
    xi = _fixed(xstar[2]) + _fixed(xstar[3])
    # powers x*^e, e = 1..d, per variable
    pr = np.empty((n, d + 1), dtype=object)
    pi = np.empty((n, d + 1), dtype=object)
    pr[:, 1], pi[:, 1] = xr, xi
    for e in range(2, d + 1):
        a, b = pr[:, e - 1], pi[:, e - 1]
        pr[:, e] = (a * xr - b * xi) >> SCALE
        pi[:, e] = (a * xi + b * xr) >> SCALE
    vr = _fixed(base.coef[0]) + _fixed(base.coef[1])
    vi = _fixed(base.coef[2]) + _fixed(base.coef[3])
    pos = base.pos.reshape(M, k)
    ex = base.exp.reshape(M, k)
    for j in range(k):
        fr, fi = pr[pos[:, j], ex[:, j]], pi[pos[:, j], ex[:, j]]
        vr, vi = (vr * fr - vi * fi) >> SCALE, (vr * fi + vi * fr) >> SCALE
    sr = vr.reshape(n, m).sum(axis=1)
    si = vi.reshape(n, m).sum(axis=1)
    # CSR with the constant appended last in each polynomial
    new_poly_start = np.arange(0, n * (m + 1) + 1, m + 1, dtype=np.int64)
    per_mono_k = np.full(n * (m + 1), k, dtype=np.int64)
    per_mono_k[m::m + 1] = 0
    new_mono_start = np.concatenate([[0], np.cumsum(per_mono_k)]).astype(np.int64)
    keep = np.ones(n * (m + 1), bool)
    keep[m::m + 1] = False
    planes = [np.zeros(n * (m + 1)) for _ in range(4)]
    for q, src in enumerate(base.coef):
        planes[q][keep] = src
    for p in range(n):
        j = p * (m + 1) + m
        planes[0][j], planes[1][j] = _to_dd(-int(sr[p]))
        planes[2][j], planes[3][j] = _to_dd(-int(si[p]))
    sys = synth.System(n, n, new_poly_start, new_mono_start, base.pos.copy(), base.exp.copy(),
                       tuple(planes), meta=dict(kind="known_root_generic", n=n, m=m, k=k,
                                                 exp_range=tuple(exp_range), seed=seed))
    return sys, xstar
