"""The library's quad-double arithmetic (qd.hpp), compiled for the host and
checked against exact rationals on the CPU.

A quad-double value is an unevaluated sum of four doubles; the tests build
operands whose words are random and non-overlapping, compute each operation
exactly in rationals, and bound the error: for sums and products relative
to the magnitudes involved (|a| + |b|, |a||b|, |a||b| + |c||d|) by a small
multiple of u^4 = 2^-212, with cancellation included.  The result must also
come back as four words of decreasing magnitude.
"""
import ctypes as C
import os
import subprocess
import tempfile
from fractions import Fraction as Fr

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1201_0499_amd", "csrc")
U4 = Fr(1, 2 ** 212)
_D = C.POINTER(C.c_double)


@pytest.fixture(scope="module")
def qp():
    d = tempfile.mkdtemp(prefix="pe_qd_")
    so = os.path.join(d, "libqd.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-ffp-contract=off",
                    "-fno-fast-math", f"-I{CSRC}", os.path.join(ROOT, "tests", "cpp", "qd_probe.cpp"),
                    "-o", so], check=True)
    L = C.CDLL(so)
    for nm in ("qp_add", "qp_mul", "qp_cmul"):
        getattr(L, nm).argtypes = [_D, _D, _D]
    L.qp_dot2.argtypes = [_D, _D, _D, _D, _D]
    L.qp_mul_d.argtypes = [_D, C.c_double, _D]
    return L


def _rand_qd(rng, scale=1.0):
    x0 = rng.uniform(-1, 1) * scale
    w = [x0]
    for _ in range(3):
        w.append(w[-1] * 2.0 ** -53 * rng.uniform(-1, 1))
    return np.array(w)


def _fr(w):
    return sum((Fr(float(v)) for v in w), Fr(0))


def _ptr(a):
    return np.ascontiguousarray(a, np.float64).ctypes.data_as(_D)


def _ordered(w):
    # words of decreasing magnitude, each below the previous one's ulp scale
    for i in range(3):
        if w[i + 1] != 0.0:
            assert abs(w[i + 1]) <= abs(w[i]) * 2.0 ** -50, w


@pytest.fixture
def rng():
    return np.random.default_rng(20240)


def test_add_and_cancellation(qp, rng):
    worst = Fr(0)
    for t in range(300):
        a = _rand_qd(rng)
        b = _rand_qd(rng, 10.0 ** rng.integers(-5, 5))
        if t % 3 == 0:  # near cancellation
            b = -a.copy()
            b[3] += a[3] * 0.5
        o = np.zeros(4)
        qp.qp_add(_ptr(a), _ptr(b), o.ctypes.data_as(_D))
        exact = _fr(a) + _fr(b)
        mag = abs(_fr(a)) + abs(_fr(b))
        worst = max(worst, abs(_fr(o) - exact) / mag)
        _ordered(o)
    assert worst <= 4 * U4, float(worst / U4)


def test_mul_and_mul_d(qp, rng):
    worst = Fr(0)
    for _ in range(300):
        a, b = _rand_qd(rng), _rand_qd(rng, 10.0 ** rng.integers(-5, 5))
        o = np.zeros(4)
        qp.qp_mul(_ptr(a), _ptr(b), o.ctypes.data_as(_D))
        worst = max(worst, abs(_fr(o) - _fr(a) * _fr(b)) / (abs(_fr(a)) * abs(_fr(b))))
        _ordered(o)
        s = float(rng.integers(1, 300))
        qp.qp_mul_d(_ptr(a), s, o.ctypes.data_as(_D))
        worst = max(worst, abs(_fr(o) - _fr(a) * Fr(s)) / (abs(_fr(a)) * Fr(s)))
    assert worst <= 16 * U4, float(worst / U4)


def test_dot2_and_complex_product_with_cancellation(qp, rng):
    worst = Fr(0)
    for t in range(200):
        a, b, c, d = (_rand_qd(rng) for _ in range(4))
        if t % 2 == 0:  # a b + c d nearly cancels
            c = -a.copy()
            d = b.copy()
            d[2] += b[2] * 1e-3
        o = np.zeros(4)
        qp.qp_dot2(_ptr(a), _ptr(b), _ptr(c), _ptr(d), o.ctypes.data_as(_D))
        exact = _fr(a) * _fr(b) + _fr(c) * _fr(d)
        M = abs(_fr(a) * _fr(b)) + abs(_fr(c) * _fr(d))
        worst = max(worst, abs(_fr(o) - exact) / M)
    assert worst <= 32 * U4, float(worst / U4)
    for _ in range(100):
        x = np.concatenate([_rand_qd(rng), _rand_qd(rng)])
        y = np.concatenate([_rand_qd(rng), _rand_qd(rng)])
        o = np.zeros(8)
        qp.qp_cmul(_ptr(x), _ptr(y), o.ctypes.data_as(_D))
        xr, xi, yr, yi = _fr(x[:4]), _fr(x[4:]), _fr(y[:4]), _fr(y[4:])
        M = abs(xr) * abs(yr) + abs(xi) * abs(yi) + abs(xr) * abs(yi) + abs(xi) * abs(yr)
        assert abs(_fr(o[:4]) - (xr * yr - xi * yi)) <= 32 * U4 * M
        assert abs(_fr(o[4:]) - (xr * yi + xi * yr)) <= 32 * U4 * M
