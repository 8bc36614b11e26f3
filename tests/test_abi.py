"""The C interface library: loads, exports every declared symbol, and
rejects invalid systems on the host (CPU only: no compute calls)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
import paper_1201_0499_amd as pe
from paper_1201_0499_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            txt = open(os.path.join(inc, fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names.update(re.findall(r"\b(pe_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_loads_and_exports_every_declared_symbol():
    L = pe.lib()
    declared = _declared()
    assert "pe_eval_jac" in declared and "pe_create_system" in declared
    missing = [n for n in sorted(declared) if not hasattr(L, n)]
    assert not missing, missing
    # the binding declares a signature for every exported entry point
    assert declared <= set(_abi.SIGNATURES), sorted(declared - set(_abi.SIGNATURES))
    assert L.pe_version().startswith(b"polyeval")


def _args(s):
    return [s.n_vars, s.n_polys, s.poly_start, s.mono_start, s.pos, s.exp, s.coef]


def _expect_einval(args, fragment):
    with pytest.raises(pe.PolyevalError) as ei:
        pe.create_system(*args)
    assert ei.value.status == 1, str(ei.value)
    assert fragment in str(ei.value)


def test_create_system_rejects_invalid_input():
    s, _ = synth.tiny_workload()
    a = _args(s)
    bad = list(a); bad[0] = 0
    _expect_einval(bad, "n_vars")
    bad = list(a); bad[1] = 0
    _expect_einval(bad, "n_polys")
    bad = list(a); bad[4] = np.where(s.pos == s.pos[1], 8, s.pos)
    _expect_einval(bad, "out of range")
    bad = list(a); p2 = s.pos.copy(); p2[0], p2[1] = p2[1], p2[0]; bad[4] = p2
    _expect_einval(bad, "strictly increasing")
    bad = list(a); e2 = s.exp.copy(); e2[5] = 0; bad[5] = e2
    _expect_einval(bad, "exponent")
    bad = list(a); e2 = s.exp.copy(); e2[5] = 257; bad[5] = e2
    _expect_einval(bad, "exponent")
    bad = list(a); c = [x.copy() for x in s.coef]; c[2][3] = np.nan; bad[6] = tuple(c)
    _expect_einval(bad, "not finite")
    bad = list(a); ps = s.poly_start.copy(); ps[-1] -= 1; bad[2] = ps
    _expect_einval(bad, "n_monos")
    bad = list(a); ps = s.poly_start.copy(); ps[3], ps[4] = ps[4], ps[3]; bad[2] = ps
    _expect_einval(bad, "decreases")


def test_null_arguments_are_rejected():
    L = pe.lib()
    assert L.pe_eval_jac(None, 1, _abi.cvec([0] * 4), _abi.cvec([0] * 4), _abi.cvec([0] * 4),
                         1, None) == 1
    assert b"NULL" in L.pe_last_error()
    assert L.pe_create_system(4, 4, 0, None, None, None, None, _abi.cvec([0] * 4), None) == 1
    assert L.pe_destroy_system(None) == 0
    assert L.pe_set_schedule(None, 1, 4, 256, 1, 0, 0) == 1
    assert L.pe_newton_qd(None, 1, None, 1e-56, 10, None, None, None, None) == 1
