"""GPU Newton corrector (pe_newton), mixed precision and all double-double,
checked against the oracle: every start must reach max_p |f_p(x)| < 1e-28
with the residual recomputed by the oracle (and in exact rationals on small
systems), converge to the known root, and report the documented statuses.
"""
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
from gpu_helpers import dev, host  # noqa: E402
from mp_known_root import known_root_system_generic  # noqa: E402

TOL = 1e-28


def _run(sys_np, starts, mode, max_iter=10, tol=TOL):
    S = pe.System.from_csr(sys_np)
    P = starts[0].shape[0]
    x = dev(starts)
    res = torch.zeros(P, dtype=torch.float64, device="cuda")
    it = torch.zeros(P, dtype=torch.int32, device="cuda")
    st = torch.zeros(P, dtype=torch.int32, device="cuda")
    code = S.newton(P, x, res, it, st, tol=tol, max_iter=max_iter, mode=mode)
    torch.cuda.synchronize()
    out = host(x), res.cpu().numpy(), it.cpu().numpy(), st.cpu().numpy(), code
    S.close()
    return out


def _oracle_residual(sys_np, x, rows):
    pts = tuple(a[rows] for a in x)
    f, _ = O.eval_dd(sys_np, pts, with_jac=False)
    return np.max(np.hypot(f[0] + f[1], f[2] + f[3]), axis=1)


@pytest.mark.parametrize("mode", [0, 1], ids=["mixed", "dd"])
def test_small_known_root_exact_residual(mode):
    n = 10
    sys_np, xstar = synth.known_root_system(n, 6, 3, (1, 3), seed=900)
    starts = synth.perturbed_starts(xstar, 4, 1e-6, seed=901)
    print(f"[case] newton small mode={mode}", flush=True)
    x, res, it, st, code = _run(sys_np, starts, mode)
    assert code == 0 and np.all(st == 0), (st, res)
    assert np.all(res < TOL) and np.all(it >= 1) and np.all(it <= 6)
    coefs = E.coefficients(sys_np)
    xs = [E.from_dd(*(a[i] for a in xstar)) for i in range(n)]
    for q in range(4):
        xq = [E.from_dd(x[0][q, i], x[1][q, i], x[2][q, i], x[3][q, i]) for i in range(n)]
        fq, _ = E.eval_exact(sys_np, xq, coefs, with_jac=False)
        assert max(v.abs_float() for v in fq) < TOL
        assert max((a - b).abs_float() for a, b in zip(xq, xs)) < 1e-26


@pytest.mark.parametrize("mode", [0, 1], ids=["mixed", "dd"])
def test_matches_oracle_newton(mode):
    """Same root as the oracle's plain dd Newton from the same starts."""
    n = 16
    sys_np, xstar = synth.known_root_system(n, 12, 4, (1, 3), seed=910)
    starts = synth.perturbed_starts(xstar, 3, 1e-6, seed=911)
    x, res, it, st, code = _run(sys_np, starts, mode)
    xo, reso, ito, sto = O.newton_dd(sys_np, starts, tol=TOL, max_iter=10)
    assert np.all(st == 0) and np.all(sto == 0)
    d = O.dd_diff_abs(x, xo)
    assert np.max(d) < 1e-26
    assert np.all(_oracle_residual(sys_np, x, np.arange(3)) < TOL)


@pytest.mark.parametrize("mode", [0, 1], ids=["mixed", "dd"])
def test_paper_scale_known_root_many_starts(mode):
    """n=128, m=256 (+1 constant), k=16, exponents 1..3, 256 starts at 1e-6
    from the root; the oracle recomputes the residual of 4 sampled starts."""
    sys_np, xstar, starts = synth.newton_workload(n_starts=256)
    print(f"[case] newton paper-scale mode={mode}", flush=True)
    x, res, it, st, code = _run(sys_np, starts, mode)
    assert code == 0 and np.all(st == 0), np.unique(st, return_counts=True)
    assert np.all(res < TOL)
    rows = np.array([0, 77, 150, 255])
    assert np.all(_oracle_residual(sys_np, x, rows) < TOL)
    err = np.max(np.hypot(x[0] + x[1] - xstar[0], x[2] + x[3] - xstar[2]))
    assert err < 1e-26
    print(f"[case] iterations: {np.bincount(it)}", flush=True)
    # quadratic convergence from 1e-6: every start needs exactly three updates
    assert np.all(it <= 3), np.bincount(it)


def test_statuses():
    n = 4
    polys = [[[(0, 1), (1, 1)], [(2, 2)], []]] * 2 + [[[(2, 1)], [(3, 1)], []], [[(3, 2)], [(0, 1)], []]]
    coefs = [[1.0, 0.5, -0.25]] * 2 + [[1.0, -1.0, 0.5], [1.0, 2.0, -1.0]]
    sing = synth.system_from_lists(n, polys, coefs)
    st0 = tuple(np.full((2, n), v) for v in (0.3, 0.0, 0.2, 0.0))
    for mode in (0, 1):
        _, res, it, st, code = _run(sing, st0, mode)
        assert code == 5 and np.all(st == 2)
    sys2, xstar = synth.known_root_system(6, 4, 2, (1, 2), seed=3)
    starts = synth.perturbed_starts(xstar, 2, 1e-3, seed=4)
    for mode in (0, 1):
        _, res, it, st, code = _run(sys2, starts, mode, max_iter=0)
        assert code == 5 and np.all(st == 1) and np.all(it == 0)
    bad = tuple(a.copy() for a in starts)
    bad[0][0, 0] = np.nan
    for mode in (0, 1):
        _, res, it, st, code = _run(sys2, bad, mode, max_iter=6)
        assert st[0] == 3 and st[1] == 0 and np.isnan(res[0])


@pytest.mark.parametrize("n,absent", [(40, 20), (100, 70), (160, 90)],
                         ids=["64-column-panels", "128-column-panels", "blocked"])
def test_zero_column_is_singular(n, absent):
    """A variable that no polynomial contains leaves its Jacobian column
    exactly zero, so the elimination meets a zero pivot at that column, in
    the middle of a panel: every start stops with status 2 (zero pivot),
    in both modes, and the call reports PE_ENOTCONVERGED."""
    polys, coefs = [], []
    for i in range(n):
        if i == absent:
            polys.append([[(0, 1), (1, 1)], []])
            coefs.append([1.0, -0.5])
        else:
            polys.append([[(i, 1)], [((i + 1) % n if (i + 1) % n != absent else (i + 2) % n, 2)], []])
            coefs.append([1.0, 0.25, -0.75])
    sys_np = synth.system_from_lists(n, polys, coefs)
    starts = tuple(np.full((3, n), v) for v in (0.4, 0.0, 0.1, 0.0))
    for mode in (0, 1):
        print(f"[case] newton zero column n={n} absent={absent} mode={mode}", flush=True)
        _, res, it, st, code = _run(sys_np, starts, mode)
        assert code == 5 and np.all(st == 2), (code, st)
        assert np.all(it == 0)


def test_rejects_non_square():
    s = synth.regular_system(6, 3, 2, (1, 2), seed=1, n_polys=4)
    S = pe.System.from_csr(s)
    x = dev(synth.points(1, 6, 2))
    z = torch.zeros(1, dtype=torch.float64, device="cuda")
    i = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(pe.PolyevalError) as ei:
        S.newton(1, x, z, i, i.clone())
    assert ei.value.status == 1
    S.close()


@pytest.mark.parametrize("mode", [0, 1], ids=["mixed", "dd"])
def test_large_known_root_sampled(mode):
    """n=512, m=1024 (+1 constant), k=32, exponents 1..5 (the large
    configuration), 8 starts at 1e-6 from the root; the oracle recomputes
    the residual of 2 of them."""
    sys_np, xstar, starts = synth.newton_large_workload(n_starts=8)
    print(f"[case] newton large mode={mode}", flush=True)
    x, res, it, st, code = _run(sys_np, starts, mode)
    assert code == 0 and np.all(st == 0), np.unique(st, return_counts=True)
    assert np.all(res < TOL)
    assert np.all(_oracle_residual(sys_np, x, np.array([0, 7])) < TOL)
    err = np.max(np.hypot(x[0] + x[1] - xstar[0], x[2] + x[3] - xstar[2]))
    assert err < 1e-26
    print(f"[case] iterations: {np.bincount(it)}", flush=True)
    assert np.all(it <= 4), np.bincount(it)


# ---------------------------------------------------------------------------
# a generic root (not a root of unity): monomial values at x* are not units
# ---------------------------------------------------------------------------

def _floor_at_root(sys_np, xstar, mode=0):
    """max_p |f_p(x*)| as the library's residual evaluates it (pe_newton with
    max_iter = 0 from x* itself), and as the oracle evaluates it."""
    pts = tuple(a.reshape(1, -1).copy() for a in xstar)
    _, res, it, st, _ = _run(sys_np, pts, mode, max_iter=0)
    return float(res[0]), float(_oracle_residual(sys_np, pts, np.array([0]))[0])


def _generic_case(sys_np, xstar, n_starts, seed, mode, max_it, tag):
    starts = synth.perturbed_starts(xstar, n_starts, 1e-6, seed=seed)
    gpu_floor, orc_floor = _floor_at_root(sys_np, xstar, mode)
    print(f"[err] newton {tag} mode={mode}: residual at x* {gpu_floor:.3e} (library), "
          f"{orc_floor:.3e} (oracle); tolerance {TOL:.0e}, margin {TOL / gpu_floor:.1f}x",
          flush=True)
    x, res, it, st, code = _run(sys_np, starts, mode)
    print(f"[case] newton {tag} mode={mode}: iterations {np.bincount(it)}, "
          f"max residual {res.max():.3e}", flush=True)
    assert code == 0 and np.all(st == 0), np.unique(st, return_counts=True)
    assert np.all(res < TOL)
    rows = np.unique(np.array([0, n_starts // 2, n_starts - 1]))
    assert np.all(_oracle_residual(sys_np, x, rows) < TOL)
    err = np.max(np.hypot((x[0] - xstar[0]) + (x[1] - xstar[1]),
                          (x[2] - xstar[2]) + (x[3] - xstar[3])))
    assert err < 1e-26, err
    assert np.all(it <= max_it), np.bincount(it)
    return gpu_floor


@pytest.mark.parametrize("mode", [0, 1], ids=["mixed", "dd"])
def test_generic_root_small_exact_residual(mode):
    """n=10 at a generic unit-circle root: the residual at the returned x is
    recomputed in exact rationals."""
    n = 10
    sys_np, xstar = known_root_system_generic(n, 6, 3, (1, 3), seed=930)
    starts = synth.perturbed_starts(xstar, 4, 1e-6, seed=931)
    x, res, it, st, code = _run(sys_np, starts, mode)
    assert code == 0 and np.all(st == 0) and np.all(res < TOL)
    coefs = E.coefficients(sys_np)
    xs = [E.from_dd(*(a[i] for a in xstar)) for i in range(n)]
    f0, _ = E.eval_exact(sys_np, xs, coefs, with_jac=False)
    assert max(v.abs_float() for v in f0) < 1e-31      # the construction
    for q in range(4):
        xq = [E.from_dd(x[0][q, i], x[1][q, i], x[2][q, i], x[3][q, i]) for i in range(n)]
        fq, _ = E.eval_exact(sys_np, xq, coefs, with_jac=False)
        assert max(v.abs_float() for v in fq) < TOL
        assert max((a - b).abs_float() for a, b in zip(xq, xs)) < 1e-26


@pytest.mark.parametrize("mode", [0, 1], ids=["mixed", "dd"])
def test_generic_root_padded_small_solver(mode):
    """n = 100 (between 65 and 127): the FP64 solve runs the 128-column
    panel elimination with 28 padding columns and a last panel of 4."""
    sys_np, xstar = known_root_system_generic(100, 24, 5, (1, 3), seed=940)
    _generic_case(sys_np, xstar, 16, 941, mode, 4, "n=100")


def test_generic_root_64_column_solver():
    """n = 50 (between 33 and 64): the 64-column panel elimination, one row
    per lane, 14 padding columns and a last panel of 2."""
    sys_np, xstar = known_root_system_generic(50, 20, 5, (1, 3), seed=945)
    _generic_case(sys_np, xstar, 16, 946, 0, 4, "n=50")


@pytest.mark.parametrize("mode", [0, 1], ids=["mixed", "dd"])
def test_generic_root_paper_scale(mode):
    """The paper-scale shape (n=128, m=256 + 1, k=16, exponents 1..3) at a
    generic root, 64 starts at 1e-6."""
    sys_np, xstar = known_root_system_generic(128, 256, 16, (1, 3), seed=950)
    floor = _generic_case(sys_np, xstar, 64, 951, mode, 4, "paper-scale")
    assert floor < TOL / 10


@pytest.fixture(scope="module")
def generic_large():
    t = __import__("time").perf_counter()
    out = known_root_system_generic(512, 1024, 32, (1, 5), seed=960)
    print(f"[case] large generic-root system built in {__import__('time').perf_counter() - t:.1f} s",
          flush=True)
    return out


@pytest.mark.parametrize("mode", [0, 1], ids=["mixed", "dd"])
def test_generic_root_large(mode, generic_large):
    """The large shape (n=512, m=1024 + 1, k=32, exponents 1..5) at a
    generic root, 8 starts at 1e-6: the residual floor at x* is printed
    with its margin to the tolerance."""
    sys_np, xstar = generic_large
    _generic_case(sys_np, xstar, 8, 961, mode, 4, "large")


# ---------------------------------------------------------------------------
# one Newton step against the oracle's solve
# ---------------------------------------------------------------------------

def _one_step(sys_np, starts, mode):
    x1, res, it, st, code = _run(sys_np, starts, mode, max_iter=1)
    assert np.all(it == 1) and np.all(st == 1), (it, st)
    return x1


@pytest.mark.parametrize("n,mode", [(128, 0), (100, 0), (65, 0), (64, 0), (50, 0), (33, 0),
                                    (160, 0), (100, 1)],
                         ids=["fp64-n128", "fp64-n100", "fp64-n65", "fp64-n64", "fp64-n50",
                              "fp64-n33", "fp64-n160-blocked", "dd-n100"])
def test_one_step_matches_oracle_solve(n, mode):
    """One update x1 = x0 - J^{-1} r against the oracle.  Mixed: J from the
    oracle's FP64 evaluator at x0 rounded to FP64, r the leading words of
    its dd residual, solved by its dd elimination; all-dd: J and r in dd.
    The step's error is bounded by a modest multiple of cond(J) times the
    working precision (n = 33 to 128: Gauss-Jordan in registers, panels
    of 8 columns, the sizes next to each kernel's bounds; n = 160: blocked
    elimination), plus the rounding of the update itself: x1 = x0 -
    step is formed in dd and rounded relative to |x1| (about 1 here), which
    in all-dd mode is larger than cond(J) u_dd |step| at |step| ~ 1e-6."""
    sys_np, xstar = synth.known_root_system(n, 12, 4, (1, 3), seed=970 + n)
    starts = synth.perturbed_starts(xstar, 3, 1e-6, seed=971 + n)
    x1 = _one_step(sys_np, starts, mode)
    rf, rJ = O.eval_dd(sys_np, starts, with_jac=(mode == 1))
    if mode == 0:
        _, (Jr, Ji) = O.eval_f64(sys_np, starts[0], starts[2])
        u = 2.0 ** -53
    else:
        u = 2.0 ** -104
    worst = 0.0
    for q in range(3):
        if mode == 0:
            A = (Jr[q].reshape(-1), np.zeros(n * n), Ji[q].reshape(-1), np.zeros(n * n))
            b = (rf[0][q], np.zeros(n), rf[2][q], np.zeros(n))
            Jc = Jr[q] + 1j * Ji[q]
        else:
            A = tuple(a[q].reshape(-1) for a in rJ)
            b = tuple(a[q] for a in rf)
            Jc = (rJ[0][q] + rJ[1][q]) + 1j * (rJ[2][q] + rJ[3][q])
        st, d = O.solve_dd(A, b)
        assert st == 0
        # |x0 - x1 - d| per coordinate, exactly in rationals
        err = 0.0
        for i in range(n):
            e = [sum((Fr(float(starts[h][q, i])) - Fr(float(x1[h][q, i])) for h in (c, c + 1)),
                     Fr(0)) - Fr(float(d[c][i])) - Fr(float(d[c + 1][i])) for c in (0, 2)]
            err = max(err, float(np.hypot(float(e[0]), float(e[1]))))
        dn = np.max(np.hypot(d[0] + d[1], d[2] + d[3]))
        xn = np.max(np.hypot(x1[0][q] + x1[1][q], x1[2][q] + x1[3][q]))
        kappa = np.linalg.cond(Jc.T)
        ratio = err / (kappa * u * dn + 2.0 ** -104 * xn)
        worst = max(worst, ratio)
    print(f"[err] one step n={n} mode={mode}: error / (cond * u * |step| + u_dd |x1|) = "
          f"{worst:.3e}", flush=True)
    assert worst < 4 * n
