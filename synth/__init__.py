"""Seeded synthetic inputs: sparse polynomial systems, evaluation points,
known-root systems and Newton starts.

This module is shared by the tests, the oracle-side checks and the bench.  It
holds no step of the evaluation method (no powers, common factors, products or
summations of monomials); it only draws random supports, exponents and unit
circle values, exactly as described below.

The paper generates its benchmark systems at random with a fixed number ``k``
of variables per monomial, a maximal exponent ``d`` per variable and a fixed
number ``m`` of monomials per polynomial (Section 2, "For establishing
benchmarks ..." and Section 4); it gives no value distribution.  The recipe
used here:

* supports: a uniform random ``k``-subset of ``{0, .., n-1}`` per monomial,
  stored in increasing order (Section 2 requires ``i_1 < i_2 < ... < i_k``);
* exponents: uniform integers in a closed range ``[e_lo, e_hi]``;
* coefficients and points: complex double-double values with a random phase
  ``theta ~ U[0, 2 pi)``; the high parts are ``(cos theta, sin theta)`` in
  FP64 and the low parts are uniform in ``(-ulp(hi)/2, ulp(hi)/2)`` so that
  every low word carries random bits.

Every generator takes an integer seed and uses numpy's PCG64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 1201049900


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def config_seed(config_index: int, replicate: int = 0) -> int:
    """Seed of replicate ``replicate`` of workload number ``config_index``."""
    return SEED_BASE + 10 * int(config_index) + int(replicate)


@dataclass
class System:
    """A sparse polynomial system ``f = (C, A)`` in CSR form.

    Polynomial ``p`` owns monomials ``poly_start[p] .. poly_start[p+1]-1``;
    monomial ``s`` owns support entries ``mono_start[s] .. mono_start[s+1]-1``
    of ``pos`` (variable index, increasing) and ``exp`` (exponent >= 1).
    ``coef`` holds four float64 planes (re_hi, re_lo, im_hi, im_lo).
    """

    n_vars: int
    n_polys: int
    poly_start: np.ndarray
    mono_start: np.ndarray
    pos: np.ndarray
    exp: np.ndarray
    coef: tuple
    meta: dict = field(default_factory=dict)

    @property
    def n_monos(self) -> int:
        return int(self.mono_start.shape[0] - 1)

    @property
    def max_k(self) -> int:
        return int(np.max(np.diff(self.mono_start))) if self.n_monos else 0

    @property
    def max_exp(self) -> int:
        return int(self.exp.max()) if self.exp.size else 0

    def monomial(self, s: int):
        a, b = int(self.mono_start[s]), int(self.mono_start[s + 1])
        return self.pos[a:b], self.exp[a:b]


def _lo_words(rng: np.random.Generator, hi: np.ndarray) -> np.ndarray:
    """Random low words with |lo| < ulp(hi)/2 (zero where hi is a power of 2)."""
    u = rng.uniform(-0.5, 0.5, size=hi.shape)
    ulp = np.spacing(np.abs(hi))
    lo = u * ulp
    mant, _ = np.frexp(np.abs(hi))
    lo[(mant == 0.5) | (hi == 0.0)] = 0.0
    return lo


def unit_circle_dd(rng: np.random.Generator, shape) -> tuple:
    """Complex double-double values with random phase on the unit circle."""
    theta = rng.uniform(0.0, 2.0 * math.pi, size=shape)
    re_hi = np.cos(theta)
    im_hi = np.sin(theta)
    re_lo = _lo_words(rng, re_hi)
    im_lo = _lo_words(rng, im_hi)
    return (re_hi, re_lo, im_hi, im_lo)


def _k_subsets(rng: np.random.Generator, n_rows: int, n: int, k: int) -> np.ndarray:
    """``n_rows`` uniform random k-subsets of range(n), each sorted."""
    if k == 0:
        return np.zeros((n_rows, 0), dtype=np.int32)
    if k > n:
        raise ValueError("k > n")
    if 2 * k > n:
        # dense case: argsort of random keys
        keys = rng.random((n_rows, n))
        out = np.sort(np.argsort(keys, axis=1)[:, :k], axis=1)
        return out.astype(np.int32)
    out = np.sort(rng.integers(0, n, size=(n_rows, k)), axis=1)
    bad = np.any(out[:, 1:] == out[:, :-1], axis=1) if k > 1 else np.zeros(n_rows, bool)
    while np.any(bad):
        idx = np.nonzero(bad)[0]
        redo = np.sort(rng.integers(0, n, size=(idx.size, k)), axis=1)
        out[idx] = redo
        bad_sub = np.any(redo[:, 1:] == redo[:, :-1], axis=1)
        bad = np.zeros(n_rows, bool)
        bad[idx[bad_sub]] = True
    return out.astype(np.int32)


def regular_system(n: int, m: int, k: int, exp_range=(1, 2), seed: int = 0,
                   n_polys: int | None = None) -> System:
    """Random system: ``n_polys`` (default n) polynomials of ``m`` monomials,
    each a product of ``k`` distinct variables raised to exponents drawn
    uniformly from ``exp_range`` (closed), with unit-circle dd coefficients."""
    rng = rng_for(seed)
    n_polys = n if n_polys is None else n_polys
    M = n_polys * m
    supp = _k_subsets(rng, M, n, k)
    lo, hi = exp_range
    exps = rng.integers(lo, hi + 1, size=(M, k)).astype(np.int32)
    coef = unit_circle_dd(rng, (M,))
    poly_start = np.arange(0, M + 1, m, dtype=np.int64)
    mono_start = np.arange(0, M * k + 1, k, dtype=np.int64) if k else np.zeros(M + 1, np.int64)
    return System(n, n_polys, poly_start, mono_start,
                  supp.reshape(-1).astype(np.int32), exps.reshape(-1),
                  coef, meta=dict(kind="regular", n=n, m=m, k=k, exp_range=tuple(exp_range), seed=seed))


def homogeneous_system(n: int, m: int, k: int, degree: int, seed: int = 0,
                       n_polys: int | None = None) -> System:
    """Random system whose every monomial has total degree ``degree``
    (k distinct variables, exponents >= 1 summing to ``degree``)."""
    if degree < k:
        raise ValueError("degree must be >= k")
    rng = rng_for(seed)
    n_polys = n if n_polys is None else n_polys
    M = n_polys * m
    supp = _k_subsets(rng, M, n, k)
    # exponents: 1 + a random composition of (degree - k) into k parts
    extra = degree - k
    exps = np.ones((M, k), dtype=np.int32)
    if extra and k:
        picks = rng.integers(0, k, size=(M, extra))
        for j in range(k):
            exps[:, j] += (picks == j).sum(axis=1).astype(np.int32)
    coef = unit_circle_dd(rng, (M,))
    poly_start = np.arange(0, M + 1, m, dtype=np.int64)
    mono_start = np.arange(0, M * k + 1, k, dtype=np.int64)
    return System(n, n_polys, poly_start, mono_start,
                  supp.reshape(-1).astype(np.int32), exps.reshape(-1), coef,
                  meta=dict(kind="homogeneous", n=n, m=m, k=k, degree=degree, seed=seed))


def points(n_points: int, n: int, seed: int) -> tuple:
    """``n_points`` unit-circle dd points, four planes of shape (n_points, n)."""
    return unit_circle_dd(rng_for(seed), (n_points, n))


def system_from_lists(n_vars: int, polys, coefs) -> System:
    """Build a System from Python lists.

    ``polys[p]`` is a list of monomials, each a list of ``(var, exp)`` pairs;
    ``coefs[p][j]`` is a complex number or a 4-tuple of planes values."""
    poly_start = [0]
    mono_start = [0]
    pos, exp = [], []
    planes = [[], [], [], []]
    for p, monos in enumerate(polys):
        for j, mono in enumerate(monos):
            for (v, e) in mono:
                pos.append(v)
                exp.append(e)
            mono_start.append(len(pos))
            c = coefs[p][j]
            if isinstance(c, tuple):
                vals = c
            else:
                c = complex(c)
                vals = (c.real, 0.0, c.imag, 0.0)
            for q in range(4):
                planes[q].append(float(vals[q]))
        poly_start.append(len(mono_start) - 1)
    return System(n_vars, len(polys), np.array(poly_start, np.int64),
                  np.array(mono_start, np.int64), np.array(pos, np.int32),
                  np.array(exp, np.int32), tuple(np.array(a, np.float64) for a in planes),
                  meta=dict(kind="lists"))


# ---------------------------------------------------------------------------
# Known-root systems and Newton starts
# ---------------------------------------------------------------------------

def _dd_round_sum(parts) -> tuple:
    """(hi, lo) with hi = RN(sum), lo = RN(sum - hi) for an exact sum of doubles."""
    hi = math.fsum(parts)
    lo = math.fsum(list(parts) + [-hi])
    return hi, lo


def known_root_system(n: int, m: int, k: int, exp_range=(1, 3), seed: int = 0,
                      coef_grid: int = 0):
    """A regular system plus one constant monomial per polynomial chosen so
    that a known point ``x*`` is a root.

    ``x*`` has coordinates drawn uniformly from the fourth roots of unity
    ``{1, i, -1, -i}``: then every monomial value ``x*^a`` is exactly a unit
    ``i^r`` and ``sum_s c_s x*^{a_s}`` is an exact sum of doubles, rounded
    once to double-double (with ``math.fsum``) for the constant term
    ``c_0 = -sum_s c_s x*^{a_s}``.  With ``coef_grid = g > 0`` the
    coefficients are first rounded to multiples of ``2^-g`` (low words
    zero), so that sum is exact in one double for ``m < 2^(52-g)`` and ``x*``
    is an exact root.  Returns ``(system, xstar_planes)``.
    """
    base = regular_system(n, m, k, exp_range, seed)
    if coef_grid:
        assert 0 < coef_grid <= 50 and m < 2 ** (52 - coef_grid)
        q = tuple(np.ldexp(np.round(np.ldexp(c, coef_grid)), -coef_grid) if i % 2 == 0
                  else np.zeros_like(c) for i, c in enumerate(base.coef))
        base = System(base.n_vars, base.n_polys, base.poly_start, base.mono_start, base.pos,
                      base.exp, q, meta=base.meta)
    rng = rng_for(seed + 7919)
    quarter = rng.integers(0, 4, size=n)            # x*_i = i**quarter[i]
    # exponent of i carried by each monomial: sum_j a_j * quarter[pos_j] (mod 4)
    M = base.n_monos
    rot = (base.exp.reshape(M, k).astype(np.int64) * quarter[base.pos.reshape(M, k)]).sum(axis=1) % 4 \
        if k else np.zeros(M, np.int64)
    crh, crl, cih, cil = base.coef
    # c * i^r, exactly (a rotation by a multiple of 90 degrees)
    rr = [crh, crl, -cih, -cil, -crh, -crl, cih, cil]
    ri = [cih, cil, crh, crl, -cih, -cil, -crh, -crl]
    vre_hi = np.choose(rot, [rr[0], rr[2], rr[4], rr[6]])
    vre_lo = np.choose(rot, [rr[1], rr[3], rr[5], rr[7]])
    vim_hi = np.choose(rot, [ri[0], ri[2], ri[4], ri[6]])
    vim_lo = np.choose(rot, [ri[1], ri[3], ri[5], ri[7]])
    # new CSR with the constant monomial appended last in each polynomial
    new_poly_start = np.arange(0, n * (m + 1) + 1, m + 1, dtype=np.int64)
    per_mono_k = np.full(n * (m + 1), k, dtype=np.int64)
    per_mono_k[m::m + 1] = 0
    new_mono_start = np.concatenate([[0], np.cumsum(per_mono_k)]).astype(np.int64)
    planes = [np.zeros(n * (m + 1)) for _ in range(4)]
    keep = np.ones(n * (m + 1), bool)
    keep[m::m + 1] = False
    for q, src in enumerate(base.coef):
        planes[q][keep] = src
    for p in range(n):
        sl = slice(p * m, (p + 1) * m)
        re_hi, re_lo = _dd_round_sum(np.concatenate([vre_hi[sl], vre_lo[sl]]).tolist())
        im_hi, im_lo = _dd_round_sum(np.concatenate([vim_hi[sl], vim_lo[sl]]).tolist())
        j = p * (m + 1) + m
        planes[0][j], planes[1][j] = -re_hi, -re_lo
        planes[2][j], planes[3][j] = -im_hi, -im_lo
    sys = System(n, n, new_poly_start, new_mono_start, base.pos.copy(), base.exp.copy(),
                 tuple(planes), meta=dict(kind="known_root", n=n, m=m, k=k,
                                           exp_range=tuple(exp_range), seed=seed,
                                           coef_grid=coef_grid))
    xs_re = np.array([1.0, 0.0, -1.0, 0.0])[quarter]
    xs_im = np.array([0.0, 1.0, 0.0, -1.0])[quarter]
    z = np.zeros(n)
    return sys, (xs_re, z.copy(), xs_im, z.copy())


def perturbed_starts(xstar, n_starts: int, scale: float, seed: int) -> tuple:
    """Starts ``x* + scale*(u + i v)`` with ``u, v ~ U[-1, 1]`` per coordinate,
    rounded once to double-double.  Planes of shape (n_starts, n)."""
    rng = rng_for(seed)
    n = xstar[0].shape[0]
    out = [np.empty((n_starts, n)) for _ in range(4)]
    for comp, (hi_idx, lo_idx) in enumerate(((0, 1), (2, 3))):
        delta = scale * rng.uniform(-1.0, 1.0, size=(n_starts, n))
        base_hi = np.broadcast_to(xstar[hi_idx], (n_starts, n))
        base_lo = np.broadcast_to(xstar[lo_idx], (n_starts, n))
        hi = base_hi + delta
        flat_h, flat_l = out[hi_idx].reshape(-1), out[lo_idx].reshape(-1)
        bh, bl, dl, hh = base_hi.reshape(-1), base_lo.reshape(-1), delta.reshape(-1), hi.reshape(-1)
        for t in range(flat_h.size):
            parts = [bh[t], bl[t], dl[t]]
            h = math.fsum(parts)
            flat_h[t] = h
            flat_l[t] = math.fsum(parts + [-h])
    return tuple(out)


# ---------------------------------------------------------------------------
# Named workloads (the benchmark shapes)
# ---------------------------------------------------------------------------

def tiny_workload(replicate: int = 0):
    """n=8, 8 polynomials of m=8 monomials with k=4 variables, exponents in
    {1,2}, one unit-circle point."""
    seed = config_seed(0, replicate)
    sys = regular_system(8, 8, 4, (1, 2), seed)
    pts = points(1, 8, seed + 1)
    return sys, pts


def paper_scale_workload(replicate: int = 0):
    """n=128, 128 polynomials of m=256 monomials with k=16 variables,
    exponents in 1..3, one unit-circle point."""
    seed = config_seed(1, replicate)
    sys = regular_system(128, 256, 16, (1, 3), seed)
    pts = points(1, 128, seed + 1)
    return sys, pts


def newton_workload(n_starts: int = 1024, n: int = 128, m: int = 256, k: int = 16,
                    exp_range=(1, 3), replicate: int = 0):
    """Known-root system (n=128, m=256 + 1 constant, k=16, exponents 1..3)
    with starts x* + 1e-6 (u + i v)."""
    seed = config_seed(2, replicate)
    sys, xstar = known_root_system(n, m, k, exp_range, seed)
    starts = perturbed_starts(xstar, n_starts, 1e-6, seed + 3)
    return sys, xstar, starts


def newton_large_workload(n_starts: int = 256, replicate: int = 0):
    """Known-root large system (n=512, m=1024 + 1 constant, k=32, exponents
    1..5) with 256 starts x* + 1e-6 (u + i v)."""
    seed = config_seed(4, replicate) + 5
    sys, xstar = known_root_system(512, 1024, 32, (1, 5), seed)
    starts = perturbed_starts(xstar, n_starts, 1e-6, seed + 3)
    return sys, xstar, starts


def batch_workload(n_systems: int = 64, points_per_system: int = 64, replicate: int = 0,
                   n_range=(16, 256), m_range=(16, 1024), k_range=(2, 16), exp_range=(1, 4)):
    """Uneven batch: per system n ~ U{16..256}, m ~ U{16..1024},
    k ~ U{2..16} (k <= n), exponents in 1..4, 64 points per system."""
    seed = config_seed(3, replicate)
    rng = rng_for(seed)
    systems, pts = [], []
    for j in range(n_systems):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        k = int(min(n, rng.integers(k_range[0], k_range[1] + 1)))
        systems.append(regular_system(n, m, k, exp_range, seed * 100 + j))
        pts.append(points(points_per_system, n, seed * 100 + 50 + j))
    return systems, pts


def large_workload(n_points: int = 256, replicate: int = 0):
    """n=512, 512 polynomials of m=1024 monomials with k=32 variables,
    exponents in 1..5, 256 unit-circle points."""
    seed = config_seed(4, replicate)
    sys = regular_system(512, 1024, 32, (1, 5), seed)
    pts = points(n_points, 512, seed + 1)
    return sys, pts


# ---------------------------------------------------------------------------
# Path tracking
# ---------------------------------------------------------------------------

def quadric_system(n: int, n_bilinear: int = 3, n_linear: int = 2, seed: int = 0) -> System:
    """Square system of quadrics: polynomial i is x_i^2 plus ``n_bilinear``
    products x_j x_k (j < k, distinct, drawn at random), ``n_linear`` linear
    terms and a constant, all with unit-circle coefficients.  With the x_i^2
    terms the leading forms have, for generic coefficients, only the trivial
    common zero: no roots at infinity, so each of the 2^n total-degree paths
    ends at one of the system's 2^n (Bezout) roots."""
    rng = rng_for(seed)
    polys, coefs = [], []
    for i in range(n):
        monos = [[(i, 2)]]
        pairs = set()
        while len(pairs) < min(n_bilinear, n * (n - 1) // 2):
            j, k = sorted(rng.choice(n, size=2, replace=False).tolist())
            pairs.add((j, k))
        monos += [[(j, 1), (k, 1)] for (j, k) in sorted(pairs)]
        lin = rng.choice(n, size=min(n_linear, n), replace=False).tolist()
        monos += [[(int(j), 1)] for j in sorted(lin)]
        monos.append([])
        th = rng.uniform(0.0, 2.0 * math.pi, size=len(monos))
        polys.append(monos)
        coefs.append([complex(math.cos(a), math.sin(a)) for a in th])
    s = system_from_lists(n, polys, coefs)
    s.meta.update(kind="quadrics", n_bilinear=n_bilinear, n_linear=n_linear, seed=seed)
    return s


def tracking_workload(n: int = 10, replicate: int = 0):
    """Quadrics in n = 10 variables (3 products, 2 linear terms and a
    constant besides x_i^2): 1024 total-degree paths, all ending at roots."""
    return quadric_system(n, 3, 2, config_seed(5, replicate))
