"""GPU Newton corrector to quad-double accuracy (pe_newton_qd): FP64
Jacobian and elimination, residual and iterate in complex quad-double.

Checked against what the mathematics fixes, not against another
implementation of the same loop:
  * systems whose coefficients lie on a 2^-40 grid have an exact root x*
    (the construction is pinned in exact rationals on the CPU); every start
    must converge to x* within 1e-58, every digit of the four words counted
    exactly;
  * at a generic root (a constant rounded to double-double, so x* is a root
    only to about 1e-32) the residual at the returned x is recomputed in
    Gaussian rationals and must be below the tolerance;
  * the register solvers (n <= 32, 32 < n <= 64, 64 < n <= 128) and the blocked
    elimination (n > 128) are each exercised, and the statuses are the
    documented ones.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

import synth
from oracle import exact as E

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1201_0499_amd as pe  # noqa: E402
from mp_known_root import known_root_system_generic  # noqa: E402

TOL = 1e-58


def _qd_starts(starts_dd):
    """dd planes -> quad-double planes (re x0..x3, im x0..x3)."""
    z = np.zeros_like(starts_dd[0])
    return [starts_dd[0], starts_dd[1], z, z.copy(), starts_dd[2], starts_dd[3], z.copy(),
            z.copy()]


def _run(sys_np, starts_dd, tol=TOL, max_iter=10):
    S = pe.System.from_csr(sys_np)
    planes = _qd_starts(starts_dd)
    P = planes[0].shape[0]
    x = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in planes]
    res = torch.zeros(P, dtype=torch.float64, device="cuda")
    it = torch.zeros(P, dtype=torch.int32, device="cuda")
    st = torch.zeros(P, dtype=torch.int32, device="cuda")
    code = S.newton_qd(P, x, res, it, st, tol=tol, max_iter=max_iter)
    torch.cuda.synchronize()
    out = [a.cpu().numpy() for a in x], res.cpu().numpy(), it.cpu().numpy(), st.cpu().numpy(), code
    S.close()
    return out


def _exact(x, row, i):
    re = sum((Fr(float(x[q][row, i])) for q in range(4)), Fr(0))
    im = sum((Fr(float(x[q][row, i])) for q in range(4, 8)), Fr(0))
    return E.GQ(re, im)


def _dist_to(x, xstar, rows):
    """max over the rows and coordinates of |x - x*|, exactly."""
    n = xstar[0].shape[0]
    worst = 0.0
    for r in rows:
        for i in range(n):
            d = _exact(x, r, i) - E.from_dd(*(a[i] for a in xstar))
            worst = max(worst, d.abs_float())
    return worst


def _exact_case(n, m, k, ex, n_starts, seed, tag, max_it=7):
    sys_np, xstar = synth.known_root_system(n, m, k, ex, seed=seed, coef_grid=40)
    starts = synth.perturbed_starts(xstar, n_starts, 1e-6, seed=seed + 1)
    print(f"[case] newton qd {tag}: n={n} m={m} k={k} starts={n_starts}", flush=True)
    x, res, it, st, code = _run(sys_np, starts)
    print(f"[case] newton qd {tag}: iterations {np.bincount(it).tolist()}, max residual "
          f"{res.max():.3e}", flush=True)
    assert code == 0 and np.all(st == 0), np.unique(st, return_counts=True)
    assert np.all(res < TOL)
    assert np.all(it >= 1) and np.all(it <= max_it), np.bincount(it)
    rows = sorted({0, n_starts // 2, n_starts - 1})
    err = _dist_to(x, xstar, rows)
    print(f"[err] newton qd {tag}: max |x - x*| {err:.3e} (bar 1e-58)", flush=True)
    assert err < 1e-58
    return sys_np, x


def test_exact_root_small():
    """n = 12 (the register solver for n <= 32); the residual at the returned
    x is also recomputed in Gaussian rationals."""
    sys_np, x = _exact_case(12, 10, 3, (1, 3), 8, 1200, "small")
    coefs = E.coefficients(sys_np)
    for r in (0, 7):
        f, _ = E.eval_exact(sys_np, [_exact(x, r, i) for i in range(12)], coefs, with_jac=False)
        worst = max(v.abs_float() for v in f)
        print(f"[err] newton qd small: exact residual of start {r}: {worst:.3e}", flush=True)
        assert worst < TOL


def test_exact_root_block_solver():
    """n = 100: the 128-column panel elimination with 28 padding columns."""
    _exact_case(100, 24, 5, (1, 3), 16, 1210, "n=100")


def test_exact_root_64_column_solver():
    """n = 50: the 64-column panel elimination, one row per lane."""
    _exact_case(50, 20, 5, (1, 3), 16, 1215, "n=50")


def test_exact_root_paper_scale():
    """The paper-scale shape (n=128, m=256 + 1, k=16, exponents 1..3), 64
    starts at 1e-6."""
    _exact_case(128, 256, 16, (1, 3), 64, 1220, "paper-scale")


def test_exact_root_blocked_elimination():
    """n = 300: the blocked elimination (FP64 panels of 16 columns)."""
    _exact_case(300, 16, 4, (1, 3), 8, 1230, "n=300")


def test_generic_root_exact_residual():
    """A generic unit-circle root whose constant is rounded to double-double:
    the residual at the returned x, in exact rationals, is below the
    tolerance, and x stays within the constant's rounding of x*."""
    n = 10
    sys_np, xstar = known_root_system_generic(n, 6, 3, (1, 3), seed=1240)
    starts = synth.perturbed_starts(xstar, 4, 1e-6, seed=1241)
    x, res, it, st, code = _run(sys_np, starts, tol=1e-56)
    print(f"[case] newton qd generic: iterations {np.bincount(it).tolist()}", flush=True)
    assert code == 0 and np.all(st == 0) and np.all(res < 1e-56)
    coefs = E.coefficients(sys_np)
    for r in range(4):
        xr = [_exact(x, r, i) for i in range(n)]
        f, _ = E.eval_exact(sys_np, xr, coefs, with_jac=False)
        worst = max(v.abs_float() for v in f)
        print(f"[err] newton qd generic: exact residual of start {r}: {worst:.3e} (bar 1e-56)",
              flush=True)
        assert worst < 1e-56
    assert _dist_to(x, xstar, range(4)) < 1e-30


def test_statuses():
    """Iteration limit 0 gives status 1 with no update; a non-finite start
    gives status 3; the call reports PE_ENOTCONVERGED (code 5)."""
    sys_np, xstar = synth.known_root_system(8, 6, 3, (1, 3), seed=1250, coef_grid=40)
    starts = synth.perturbed_starts(xstar, 2, 1e-6, seed=1251)
    x, res, it, st, code = _run(sys_np, starts, max_iter=0)
    assert code == 5 and np.all(st == 1) and np.all(it == 0)
    bad = tuple(a.copy() for a in starts)
    bad[0][1, 3] = np.nan
    x, res, it, st, code = _run(sys_np, bad)
    assert code == 5 and st[0] == 0 and st[1] == 3


def test_power_table_that_does_not_fit_is_refused():
    """n = 512 with exponents up to 5: the quad-double table (64 bytes per
    entry) exceeds 160 KiB of LDS."""
    sys_np, xstar = synth.known_root_system(512, 4, 2, (5, 5), seed=1260)
    starts = synth.perturbed_starts(xstar, 1, 1e-6, seed=1261)
    with pytest.raises(pe.PolyevalError) as ei:
        _run(sys_np, starts)
    assert ei.value.status == 4 and "power table" in str(ei.value)
