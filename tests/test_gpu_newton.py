"""GPU Newton corrector (pe_newton), mixed precision and all double-double,
checked against the oracle: every start must reach max_p |f_p(x)| < 1e-28
with the residual recomputed by the oracle (and in exact rationals on small
systems), converge to the known root, and report the documented statuses.
"""
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
    xs = np.stack([xstar[0], xstar[2]])
    err = np.max(np.hypot(x[0] + x[1] - xstar[0], x[2] + x[3] - xstar[2]))
    assert err < 1e-26
    print(f"[case] iterations: {np.bincount(it)}", flush=True)


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
