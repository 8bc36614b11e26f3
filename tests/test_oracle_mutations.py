"""The oracle's pins catch plausible mistakes (CPU only).

Each case plants one mistake in a copy of the oracle's C source (a dropped
term, a wrong sign, a transposed index, a lost error term ...), builds it
into a temporary library, and checks that at least one pin of
``test_oracle_pins`` fails against it.  The real oracle is restored after.
"""
import os
import shutil
import tempfile

import pytest

import synth
from oracle import build as OB
from oracle import ddoracle as O

import test_oracle_pins as PINS

MUTATIONS = {
    "drop_last_monomial": ("s < poly_start[p + 1]; ++s) {\n            int64_t b = mono_start[s], e = mono_start[s + 1];\n            ocdd c = load_cdd(coef, s);",
                           "s < poly_start[p + 1] - 1; ++s) {\n            int64_t b = mono_start[s], e = mono_start[s + 1];\n            ocdd c = load_cdd(coef, s);"),
    "complex_mul_sign": ("r.re = o_add(o_mul(a.re, b.re), o_neg(o_mul(a.im, b.im)));",
                         "r.re = o_add(o_mul(a.re, b.re), o_mul(a.im, b.im));"),
    "exponent_factor_dropped": ("ocdd d = c_scale(c, (double)expo[j]);", "ocdd d = c;"),
    "jacobian_transposed": ("int64_t at = (int64_t)pos[j] * n_polys + p;\n                J_col[at]",
                            "int64_t at = (int64_t)p * n_polys + pos[j];\n                J_col[at]"),
    "derivative_power_off_by_one": ("int32_t times = expo[l] - (l == j ? 1 : 0);\n                    for (int32_t r = 0; r < times; ++r)\n                        d = c_mul(d, x[pos[l]]);",
                                    "int32_t times = expo[l] - (l == j ? 0 : 0);\n                    for (int32_t r = 0; r < times; ++r)\n                        d = c_mul(d, x[pos[l]]);"),
    "dd_mul_cross_term_dropped": ("double c2 = t1 + t2;", "double c2 = t1;"),
    "two_sum_error_half": ("double e = (a - (s - bb)) + (b - bb);", "double e = (a - (s - bb));"),
    "dd_add_low_sum_dropped": ("double w = t.lo + v.lo;", "double w = v.lo;"),
    "coefficient_conjugated": ("ocdd c = load_cdd(coef, s);\n            /* value",
                               "ocdd c = load_cdd(coef, s);\n            c.im.hi = -c.im.hi; c.im.lo = -c.im.lo;\n            /* value"),
    "newton_update_sign": ("xp[i] = c_sub(xp[i], dx[i]);", "xp[i] = c_add(xp[i], dx[i]);"),
    # magnitude scales of the error metric
    "scale_derivative_exponent_not_reduced": (
        "d *= pow(ax[pos[l]], (double)(expo[l] - (l == j ? 1 : 0)));",
        "d *= pow(ax[pos[l]], (double)(expo[l]));"),
    "scale_exponent_factor_squared": ("double d = c * (double)expo[j];",
                                      "double d = c * (double)expo[j] * (double)expo[j];"),
    "scale_value_power_off_by_one": ("v *= pow(ax[pos[j]], (double)expo[j]);",
                                     "v *= pow(ax[pos[j]], (double)(expo[j] - 1));"),
    "scale_coefficient_modulus_dropped": ("double c = hypot(coef_re[s], coef_im[s]);",
                                          "double c = 1.0;"),
}


def _pins():
    sys_t, pts_t = synth.tiny_workload()
    return [
        lambda: PINS.test_two_sum_and_two_prod_are_error_free(),
        lambda: PINS.test_dd_add_mul_div_error_bounds(),
        lambda: PINS.test_dd_oracle_matches_exact_on_tiny_workload(),
        lambda: PINS.test_dd_oracle_matches_exact_on_special_cases(),
        lambda: PINS.test_dd_oracle_euler_identity_medium(),
        lambda: PINS.test_dd_oracle_derivative_identity_medium(),
        lambda: PINS.test_dd_newton_converges_to_known_root(0),
        lambda: PINS.test_scales_are_the_magnitude_system_at_the_modulus_point(71),
        lambda: PINS.test_scales_euler_identity_homogeneous(),
        lambda: PINS.test_scales_equal_the_values_for_positive_data(),
    ]


@pytest.fixture(scope="module")
def workdir():
    d = tempfile.mkdtemp(prefix="orc_mut_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, workdir):
    old, new = MUTATIONS[name]
    src = open(OB.SRC).read()
    assert src.count(old) == 1, name
    mutated = os.path.join(workdir, f"{name}.c")
    with open(mutated, "w") as fh:
        fh.write(src.replace(old, new))
    lib = os.path.join(workdir, f"lib{name}.so")
    import subprocess
    subprocess.run(["gcc", *OB.CFLAGS, "-o", lib, mutated, "-lm"], check=True)
    import ctypes
    saved = O._LIB
    try:
        O._LIB = None
        real = OB.LIB
        OB.LIB = lib
        OB_SRC = OB.SRC
        OB.SRC = mutated
        caught = []
        for pin in _pins():
            try:
                pin()
            except (AssertionError, ValueError, ZeroDivisionError, OverflowError):
                caught.append(True)
                break
        assert caught, f"no pin caught mutation {name}"
    finally:
        OB.LIB = real
        OB.SRC = OB_SRC
        O._LIB = saved
