"""GPU parity of pe_eval_jac_qd (complex quad-double) against the exact
evaluation in Gaussian rationals (oracle/exact.py), on systems small enough
for exact arithmetic and on one polynomial of the paper-scale system.

Bar: each output within 1e-58 of the exact value, relative to the sum of
the magnitudes of its terms (the condition scale of the other parity
tests).  Each complex quad-double operation errs by at most about 32 u^4
of the magnitudes involved (u^4 = 2^-212 ~ 1.5e-64, tests/test_qd_host.py);
an output of a monomial of k variables goes through about 2k products and
one sum per term, so k <= 16 stays near 1e-61 of the scale, which the bar
clears with room.  Double-double cannot meet it (its bar is 1e-28)."""
from fractions import Fraction as Fr

import numpy as np
import pytest

import synth
from oracle import ddoracle as O
from oracle import exact as E

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1201_0499_amd as pe  # noqa: E402

BAR = 1e-58


def _qd_points(P, n, seed):
    """dd unit-circle points with two more random words per component."""
    hi = synth.points(P, n, seed)
    rng = synth.rng_for(seed + 17)
    planes = []
    for re_or_im in (0, 2):
        x0, x1 = hi[re_or_im], hi[re_or_im + 1]
        x2 = x1 * 2.0 ** -53 * rng.uniform(-1, 1, size=x1.shape)
        x3 = x2 * 2.0 ** -53 * rng.uniform(-1, 1, size=x1.shape)
        planes += [x0, x1, x2, x3]
    return planes  # re x0..x3, im x0..x3


def _gq(planes, idx):
    re = sum((Fr(float(planes[q][idx])) for q in range(4)), Fr(0))
    im = sum((Fr(float(planes[q][idx])) for q in range(4, 8)), Fr(0))
    return E.GQ(re, im)


def _run(sys_np, planes):
    P, n = planes[0].shape
    S = pe.System.from_csr(sys_np)
    x = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in planes]
    f = [torch.full((P, sys_np.n_polys), float("nan"), dtype=torch.float64, device="cuda")
         for _ in range(8)]
    J = [torch.full((P, n, sys_np.n_polys), float("nan"), dtype=torch.float64, device="cuda")
         for _ in range(8)]
    S.eval_jac_qd(P, x, f, J)
    torch.cuda.synchronize()
    S.close()
    return [a.cpu().numpy() for a in f], [a.cpu().numpy() for a in J]


def _subsystem(sys_np, polys):
    """The polynomials `polys` of a system, as a system of their own."""
    ps, ms, pos, ex, coef = [0], [0], [], [], [[] for _ in range(4)]
    for p in polys:
        for s in range(int(sys_np.poly_start[p]), int(sys_np.poly_start[p + 1])):
            a, b = int(sys_np.mono_start[s]), int(sys_np.mono_start[s + 1])
            pos += list(sys_np.pos[a:b])
            ex += list(sys_np.exp[a:b])
            ms.append(len(pos))
            for q in range(4):
                coef[q].append(float(sys_np.coef[q][s]))
        ps.append(len(ms) - 1)
    return synth.System(sys_np.n_vars, len(polys), np.array(ps, np.int64), np.array(ms, np.int64),
                        np.array(pos, np.int32), np.array(ex, np.int32),
                        tuple(np.array(c, np.float64) for c in coef), meta=dict(kind="sub"))


def _check(sys_np, planes, polys=None, tag="", points=None):
    P, n = planes[0].shape
    print(f"[case] qd {tag} n={n} M={sys_np.n_monos} P={P}", flush=True)
    f, J = _run(sys_np, planes)
    polys = list(range(sys_np.n_polys)) if polys is None else list(polys)
    sub = _subsystem(sys_np, polys)
    dd_pts = (planes[0], planes[1], planes[4], planes[5])
    Sf, SJ = O.scales(sys_np, dd_pts[0], dd_pts[2])
    worst = 0.0
    for pt in (range(P) if points is None else points):
        x = [_gq(planes, (pt, i)) for i in range(n)]
        ef, eJ = E.eval_exact(sub, x)
        for k, p in enumerate(polys):
            ef_p, eJ_p = ef[k], eJ[k]
            got = _gq(f, (pt, p))
            d = abs(got.re - ef_p.re) + abs(got.im - ef_p.im)
            worst = max(worst, float(d) / Sf[pt, p] if Sf[pt, p] > 0 else float(d))
            for i in range(n):
                got = _gq(J, (pt, i, p))
                if SJ[pt, i, p] == 0:
                    assert all(J[q][pt, i, p] == 0.0 for q in range(8))
                    continue
                d = abs(got.re - eJ_p[i].re) + abs(got.im - eJ_p[i].im)
                worst = max(worst, float(d) / SJ[pt, i, p])
    print(f"[err] qd {tag}: worst scaled error {worst:.3e} (bar {BAR:.0e})", flush=True)
    assert worst < BAR, worst
    return worst


def test_tiny_and_ragged_exact():
    sys_np, _ = synth.tiny_workload()
    _check(sys_np, _qd_points(2, sys_np.n_vars, 3), tag="tiny")
    sys_np = synth.regular_system(20, 37, 4, (1, 3), seed=7, n_polys=11)
    _check(sys_np, _qd_points(2, 20, 8), tag="ragged")


def test_split_polynomials_exact():
    """Few (polynomial, point) pairs: six polynomials of 800 monomials at one
    point run on four workgroups each (four chunks of 256 monomials, the
    last short), whose partial rows the combination kernel adds; the same
    system at 48 points takes one workgroup per polynomial and point."""
    sys_np = synth.regular_system(24, 800, 4, (1, 3), seed=11, n_polys=6)
    _check(sys_np, _qd_points(1, 24, 12), polys=[0, 5], tag="split G=4")
    _check(sys_np, _qd_points(48, 24, 13), polys=[2], tag="G=1, 48 points", points=[0, 47])


def test_special_cases_exact():
    polys = [
        [[], [(0, 1)], [(1, 2), (3, 1)], [(0, 5), (2, 8)]],
        [[(0, 1), (1, 1), (2, 1), (3, 1)], [(0, 1), (1, 1), (2, 1), (3, 1)], [(2, 3)]],
        [],
        [[(1, 1), (2, 2)], [(4, 6)], []],
        [[(0, 2), (1, 3), (2, 1), (3, 2), (4, 1)]],
    ]
    rng = synth.rng_for(1234)
    coefs = []
    for monos in polys:
        pl = synth.unit_circle_dd(rng, (max(1, len(monos)),))
        coefs.append([tuple(float(a[j]) for a in pl) for j in range(len(monos))])
    sys_np = synth.system_from_lists(5, polys, coefs)
    _check(sys_np, _qd_points(3, 5, 55), tag="special")


def test_paper_scale_one_polynomial_exact():
    sys_np, _ = synth.paper_scale_workload()
    _check(sys_np, _qd_points(1, sys_np.n_vars, 91), polys=[77], tag="paper scale")


def test_values_only_match_full_call():
    """out_J = NULL on the paper-scale system at one point (each polynomial
    split over two workgroups): f is bit for bit the f of the call with the
    Jacobian, and no Jacobian plane is touched."""
    sys_np, _ = synth.paper_scale_workload()
    planes = _qd_points(1, sys_np.n_vars, 92)
    f_full, _ = _run(sys_np, planes)
    S = pe.System.from_csr(sys_np)
    x = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in planes]
    f = [torch.full((1, sys_np.n_polys), float("nan"), dtype=torch.float64, device="cuda")
         for _ in range(8)]
    S.eval_jac_qd(1, x, f, None)
    torch.cuda.synchronize()
    S.close()
    for q in range(8):
        assert np.array_equal(f[q].cpu().numpy().view(np.int64), f_full[q].view(np.int64)), q

