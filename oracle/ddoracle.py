"""ORACLE -- test infrastructure only.

ctypes front end of the plain C evaluator in ``ddeval.c``: the definition of
``f`` and its Jacobian (Section 2, equation (1)) in complex double-double and
in complex FP64, magnitude scales for a condition-scaled error, a dense dd
solver and a plain dd Newton corrector.  Arrays follow the same layouts as the
GPU library: points ``[P][n]``, values ``[P][n_polys]``, Jacobians
``[P][n][n_polys]`` (column-major per point), one float64 array per plane
``(re_hi, re_lo, im_hi, im_lo)``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None
_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)
_I32 = C.POINTER(C.c_int32)
_P4 = _D * 4


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build(force=True)
        L = C.CDLL(path)
        L.orc_two_sum.argtypes = [C.c_double, C.c_double, _D, _D]
        L.orc_two_prod.argtypes = [C.c_double, C.c_double, _D, _D]
        for nm in ("orc_dd_add", "orc_dd_mul", "orc_dd_div"):
            getattr(L, nm).argtypes = [C.c_double] * 4 + [_D, _D]
        L.orc_eval_dd.argtypes = [C.c_int32, C.c_int32, _I64, _I64, _I32, _I32, _P4, C.c_int64,
                                  _P4, _P4, C.c_void_p, _I32, C.c_int32]
        L.orc_eval_f64.argtypes = [C.c_int32, C.c_int32, _I64, _I64, _I32, _I32, _D, _D,
                                   C.c_int64, _D, _D, _D, _D, _D, _D, _I32, C.c_int32]
        L.orc_eval_dd_fast.argtypes = [C.c_int32, C.c_int32, _I64, _I64, _I32, _I32, _P4,
                                       C.c_int64, _P4, _P4, C.c_void_p, _I32, C.c_int32,
                                       C.c_int32, _I32]
        L.orc_scales.argtypes = [C.c_int32, C.c_int32, _I64, _I64, _I32, _I32, _D, _D,
                                 C.c_int64, _D, _D, _D, _D, _I32, C.c_int32]
        L.orc_solve_dd.argtypes = [C.c_int32, _P4, _P4, _P4]
        L.orc_newton_dd.argtypes = [C.c_int32, _I64, _I64, _I32, _I32, _P4, C.c_int64, _P4,
                                    C.c_double, C.c_int32, _D, _I32, _I32]
        for nm in ("orc_eval_dd", "orc_eval_f64", "orc_scales", "orc_solve_dd", "orc_newton_dd",
                   "orc_eval_dd_fast"):
            getattr(L, nm).restype = C.c_int
        _LIB = L
    return _LIB


def _ptr(a, ct=_D):
    return a.ctypes.data_as(ct)


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _planes(planes):
    arrs = [_c64(a) for a in planes]
    return arrs, _P4(*[_ptr(a) for a in arrs])


def _sys_args(system):
    ps = np.ascontiguousarray(system.poly_start, np.int64)
    ms = np.ascontiguousarray(system.mono_start, np.int64)
    pos = np.ascontiguousarray(system.pos, np.int32)
    ex = np.ascontiguousarray(system.exp, np.int32)
    return (ps, ms, pos, ex), (_ptr(ps, _I64), _ptr(ms, _I64), _ptr(pos, _I32), _ptr(ex, _I32))


# ---------------------------------------------------------------------------
# primitives
# ---------------------------------------------------------------------------

def two_sum(a: float, b: float):
    s, e = C.c_double(), C.c_double()
    lib().orc_two_sum(a, b, C.byref(s), C.byref(e))
    return s.value, e.value


def two_prod(a: float, b: float):
    p, e = C.c_double(), C.c_double()
    lib().orc_two_prod(a, b, C.byref(p), C.byref(e))
    return p.value, e.value


def _dd2(fn, x, y):
    zh, zl = C.c_double(), C.c_double()
    fn(x[0], x[1], y[0], y[1], C.byref(zh), C.byref(zl))
    return zh.value, zl.value


def dd_add(x, y):
    return _dd2(lib().orc_dd_add, x, y)


def dd_mul(x, y):
    return _dd2(lib().orc_dd_mul, x, y)


def dd_div(x, y):
    return _dd2(lib().orc_dd_div, x, y)


# ---------------------------------------------------------------------------
# evaluation
# ---------------------------------------------------------------------------

def eval_dd(system, x_planes, with_jac: bool = True, polys=None):
    """Definitional complex-dd values (and Jacobians) at every point.

    Returns ``(f_planes, J_planes)``; with ``polys`` only those polynomials are
    computed (other entries are NaN)."""
    n, npoly = system.n_vars, system.n_polys
    xs, xp = _planes(x_planes)
    P = xs[0].size // n
    f = [np.full((P, npoly), np.nan) for _ in range(4)]
    fp = _P4(*[_ptr(a) for a in f])
    if with_jac:
        J = [np.full((P, n, npoly), np.nan) for _ in range(4)]
        Jarr = _P4(*[_ptr(a) for a in J])
        Jp = C.cast(Jarr, C.c_void_p)
    else:
        J, Jp = None, None
    keep, sargs = _sys_args(system)
    cs, cp = _planes(system.coef)
    if polys is None:
        sel, selp, nsel = None, None, 0
    else:
        sel = np.ascontiguousarray(polys, np.int32)
        selp, nsel = _ptr(sel, _I32), int(sel.size)
    rc = lib().orc_eval_dd(n, npoly, *sargs, cp, P, xp, fp, Jp, selp, nsel)
    assert rc == 0
    return tuple(f), (tuple(J) if J is not None else None)


def _selection(polys):
    if polys is None:
        return None, None, 0
    sel = np.ascontiguousarray(polys, np.int32)
    return sel, _ptr(sel, _I32), int(sel.size)


def eval_f64(system, x_re, x_im, with_jac: bool = True, polys=None):
    """Definitional complex-FP64 values and Jacobians (real/imag arrays);
    with ``polys`` only those polynomials are computed (others are NaN)."""
    n, npoly = system.n_vars, system.n_polys
    xr, xi = _c64(x_re), _c64(x_im)
    P = xr.size // n
    fr, fi = np.full((P, npoly), np.nan), np.full((P, npoly), np.nan)
    if with_jac:
        Jr, Ji = np.full((P, n, npoly), np.nan), np.full((P, n, npoly), np.nan)
        Jrp, Jip = _ptr(Jr), _ptr(Ji)
    else:
        Jr = Ji = None
        Jrp = Jip = None
    keep, sargs = _sys_args(system)
    cr, ci = _c64(system.coef[0]), _c64(system.coef[2])
    sel, selp, nsel = _selection(polys)
    rc = lib().orc_eval_f64(n, npoly, *sargs, _ptr(cr), _ptr(ci), P, _ptr(xr), _ptr(xi),
                            _ptr(fr), _ptr(fi), Jrp, Jip, selp, nsel)
    assert rc == 0
    return (fr, fi), ((Jr, Ji) if with_jac else None)


def eval_dd_fast(system, x_planes, with_jac: bool = True, polys=None, threads: int = 0):
    """The same complex-dd values and Jacobians by the fast mode (power
    table, common factor, prefix/suffix products; OpenMP over (point,
    polynomial) pairs, ``threads`` = 0: OpenMP's default).  Returns
    ``(f_planes, J_planes, threads_used)``."""
    n, npoly = system.n_vars, system.n_polys
    xs, xp = _planes(x_planes)
    P = xs[0].size // n
    f = [np.full((P, npoly), np.nan) for _ in range(4)]
    fp = _P4(*[_ptr(a) for a in f])
    if with_jac:
        J = [np.full((P, n, npoly), np.nan) for _ in range(4)]
        Jp = C.cast(_P4(*[_ptr(a) for a in J]), C.c_void_p)
    else:
        J, Jp = None, None
    keep, sargs = _sys_args(system)
    cs, cp = _planes(system.coef)
    sel, selp, nsel = _selection(polys)
    used = C.c_int32(0)
    rc = lib().orc_eval_dd_fast(n, npoly, *sargs, cp, P, xp, fp, Jp, selp, nsel, int(threads),
                                C.byref(used))
    assert rc == 0
    return tuple(f), (tuple(J) if J is not None else None), int(used.value)


def scales(system, x_re, x_im, with_jac: bool = True, polys=None):
    """Condition scales ``Sf[P][n_polys]`` and ``SJ[P][n][n_polys]``:
    sums of magnitudes of the terms that make up each output."""
    n, npoly = system.n_vars, system.n_polys
    xr, xi = _c64(x_re), _c64(x_im)
    P = xr.size // n
    Sf = np.full((P, npoly), np.nan)
    SJ = np.full((P, n, npoly), np.nan) if with_jac else None
    keep, sargs = _sys_args(system)
    cr, ci = _c64(system.coef[0]), _c64(system.coef[2])
    if polys is None:
        sel, selp, nsel = None, None, 0
    else:
        sel = np.ascontiguousarray(polys, np.int32)
        selp, nsel = _ptr(sel, _I32), int(sel.size)
    rc = lib().orc_scales(n, npoly, *sargs, _ptr(cr), _ptr(ci), P, _ptr(xr), _ptr(xi),
                          _ptr(Sf), _ptr(SJ) if with_jac else None, selp, nsel)
    assert rc == 0
    return Sf, SJ


def solve_dd(A_planes, b_planes):
    """Solve ``A x = b`` (complex dd, A column-major n x n) by Gaussian
    elimination with partial pivoting.  Returns ``(status, x_planes)``."""
    A = [np.array(a, dtype=np.float64, order="C").reshape(-1).copy() for a in A_planes]
    b = [np.array(v, dtype=np.float64).reshape(-1).copy() for v in b_planes]
    n = b[0].size
    x = [np.zeros(n) for _ in range(4)]
    st = lib().orc_solve_dd(n, _P4(*[_ptr(a) for a in A]), _P4(*[_ptr(a) for a in b]),
                            _P4(*[_ptr(a) for a in x]))
    return st, tuple(x)


def newton_dd(system, x0_planes, tol: float = 1e-28, max_iter: int = 8):
    """Plain dd Newton from every start.  Returns (x_planes, res, iters, status)."""
    if system.n_vars != system.n_polys:
        raise ValueError("Newton needs a square system")
    n = system.n_vars
    xs = [np.array(a, dtype=np.float64).copy() for a in x0_planes]
    S = xs[0].size // n
    res = np.zeros(S)
    iters = np.zeros(S, np.int32)
    status = np.zeros(S, np.int32)
    keep, sargs = _sys_args(system)
    cs, cp = _planes(system.coef)
    lib().orc_newton_dd(n, *sargs, cp, S, _P4(*[_ptr(a) for a in xs]), float(tol),
                        int(max_iter), _ptr(res), _ptr(iters, _I32), _ptr(status, _I32))
    return tuple(a.reshape(S, n) for a in xs), res, iters, status


# ---------------------------------------------------------------------------
# error metric
# ---------------------------------------------------------------------------

def dd_diff_abs(a_planes, b_planes):
    """|a - b| for complex dd arrays given as planes, accurate to a few ulps of
    the difference (the differences of hi and lo words are combined in FP64,
    which is exact enough for differences far below |a|)."""
    dre = (a_planes[0] - b_planes[0]) + (a_planes[1] - b_planes[1])
    dim = (a_planes[2] - b_planes[2]) + (a_planes[3] - b_planes[3])
    return np.hypot(dre, dim)
