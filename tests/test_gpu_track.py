"""GPU path tracker (pe_start_solutions, pe_track) against the oracle's
tracker (oracle/tracker.py), which follows the same rules on the CPU.

Parity is per path: the same start, tracked by both, must reach the same
root (end points compared after the double-double endgame on both sides)
or fail on both; every end point the GPU reports as converged must have a
residual below 1e-28 recomputed by the oracle's dd evaluator.  Step counts
and the kind of failure of a diverging path (step underflow, zero pivot,
non-finite values, step limit) may differ, since the step decisions are
taken on FP64 solutions that round differently, so they are not compared.
"""
import numpy as np
import pytest

import synth
from oracle import ddoracle as O
from oracle import tracker as TR

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1201_0499_amd as pe  # noqa: E402
from gpu_helpers import host  # noqa: E402

GAMMA = 0.6 + 0.8j


def _gpu_track(sys_np, P, first=0, **params):
    S = pe.System.from_csr(sys_np)
    n = sys_np.n_vars
    x = tuple(torch.full((P, n), float("nan"), dtype=torch.float64, device="cuda") for _ in range(4))
    S.start_solutions(first, P, x)
    torch.cuda.synchronize()
    x_start = host(x)
    t = torch.zeros(P, dtype=torch.float64, device="cuda")
    res = torch.zeros(P, dtype=torch.float64, device="cuda")
    steps = torch.zeros(P, dtype=torch.int32, device="cuda")
    st = torch.zeros(P, dtype=torch.int32, device="cuda")
    code = S.track(P, x, t, steps, st, res, gamma=GAMMA, **params)
    torch.cuda.synchronize()
    out = dict(x0=x_start, x=host(x), t=t.cpu().numpy(), steps=steps.cpu().numpy(),
               status=st.cpu().numpy(), res=res.cpu().numpy(), code=code)
    S.close()
    return out


def _residual(sys_np, planes, rows):
    f, _ = O.eval_dd(sys_np, tuple(a[rows] for a in planes), with_jac=False)
    return np.hypot(f[0] + f[1], f[2] + f[3]).max(axis=1)


def _compare(sys_np, P, tol=1e-24, **params):
    print(f"[case] track n={sys_np.n_vars} paths={P} params={params}", flush=True)
    g = _gpu_track(sys_np, P, **params)
    x0 = TR.start_solutions(sys_np, 0, P)
    # start solutions: the GPU's against the oracle's
    assert np.max(np.abs(g["x0"][0] + 1j * g["x0"][2] - x0)) < 1e-15
    assert np.all(g["x0"][1] == 0) and np.all(g["x0"][3] == 0)
    planes, T, steps, status, res = TR.track(sys_np, x0, gamma=GAMMA, **params)
    assert np.array_equal(g["status"] == 0, status == 0), (g["status"], status)
    ok = np.nonzero(status == 0)[0]
    assert np.all(g["t"][ok] == 1.0)
    if ok.size:
        d = np.max(np.abs((g["x"][0][ok] + g["x"][1][ok]) - (planes[0][ok] + planes[1][ok])) +
                   np.abs((g["x"][2][ok] + g["x"][3][ok]) - (planes[2][ok] + planes[3][ok])))
        assert d < tol, d
        assert np.max(_residual(sys_np, g["x"], ok)) < 1e-28
        assert np.max(g["res"][ok]) < 1e-28
    return g


def test_decoupled_squares():
    rng = synth.rng_for(21)
    n = 3
    c = np.exp(2j * np.pi * rng.uniform(size=n)) * rng.uniform(0.5, 2.0, size=n)
    s = synth.system_from_lists(n, [[[(i, 2)], []] for i in range(n)],
                                [[1.0, -complex(c[i])] for i in range(n)])
    g = _compare(s, 8)
    assert g["code"] == 0


def test_univariate_degree_five():
    rng = synth.rng_for(31)
    coef = np.exp(2j * np.pi * rng.uniform(size=6))
    s = synth.system_from_lists(1, [[[(0, e)] if e else [] for e in range(6)]],
                                [[complex(v) for v in coef]])
    g = _compare(s, 5)
    got = np.sort_complex(g["x"][0][:, 0] + 1j * g["x"][2][:, 0])
    assert np.max(np.abs(got - np.sort_complex(np.roots(coef[::-1])))) < 1e-9


@pytest.mark.parametrize("n", [2, 4, 5])
def test_quadrics_every_path(n):
    s = synth.quadric_system(n, 2, 2, seed=60 + n)
    g = _compare(s, 2 ** n)
    assert g["code"] == 0
    X = g["x"][0] + 1j * g["x"][2]
    dist = np.abs(X[:, None, :] - X[None, :, :]).max(axis=2) + np.eye(2 ** n)
    assert dist.min() > 1e-6


def test_root_at_infinity_and_without_endgame():
    s = synth.system_from_lists(1, [[[(0, 2)], [(0, 1)], []]], [[0.0, 1.0, -0.5]])
    g = _compare(s, 2, max_steps=400)
    assert g["code"] == 5 and np.sum(g["status"] == 0) == 1
    # no endgame: FP64 end points, NaN residuals
    g2 = _gpu_track(s, 2, max_steps=400, end_tol=0.0)
    ok = g2["status"] == 0
    assert np.all(np.isnan(g2["res"]))
    assert abs(g2["x"][0][ok][0, 0] - 0.5) < 1e-9


def test_tracking_workload_sample():
    """The tracking workload (quadrics, n = 10, 1024 paths): every path
    reaches a root, the 1024 roots are distinct, and 16 sampled paths match
    the oracle's tracker."""
    s = synth.tracking_workload()
    print("[case] tracking workload n=10 paths=1024", flush=True)
    g = _gpu_track(s, 1024)
    assert g["code"] == 0 and np.all(g["status"] == 0)
    X = g["x"][0] + 1j * g["x"][2]
    key = np.round(X / 1e-6).astype(np.complex128)
    assert len({tuple(r) for r in key}) == 1024
    rows = np.arange(0, 1024, 64)
    assert np.max(_residual(s, g["x"], rows)) < 1e-28
    planes, T, steps, status, res = TR.track(s, TR.start_solutions(s, 0, 1024)[rows], gamma=GAMMA)
    assert np.all(status == 0)
    d = np.max(np.abs(X[rows] - (planes[0] + 1j * planes[2])))
    assert d < 1e-12, d


def test_invalid_arguments():
    s = synth.regular_system(4, 3, 2, (1, 2), seed=3, n_polys=3)  # not square
    S = pe.System.from_csr(s)
    x = tuple(torch.zeros((2, 4), dtype=torch.float64, device="cuda") for _ in range(4))
    with pytest.raises(pe.PolyevalError):
        S.start_solutions(0, 2, x)
    S.close()
    const = synth.system_from_lists(2, [[[(0, 1)], []], [[]]], [[1.0, 1.0], [2.0]])
    S = pe.System.from_csr(const)
    with pytest.raises(pe.PolyevalError):  # polynomial 1 has degree 0
        S.start_solutions(0, 2, x)
    S.close()
    q = synth.quadric_system(2, 1, 1, seed=5)
    S = pe.System.from_csr(q)
    t = torch.zeros(2, dtype=torch.float64, device="cuda")
    st = torch.zeros(2, dtype=torch.int32, device="cuda")
    x2 = tuple(torch.zeros((2, 2), dtype=torch.float64, device="cuda") for _ in range(4))
    for bad in (dict(h_init=0.0), dict(h_min=1.0), dict(corr_iters=0), dict(gamma=0.0),
                dict(max_steps=0), dict(end_tol=-1.0)):
        with pytest.raises(pe.PolyevalError):
            S.track(2, x2, t, st, st, t, **bad)
    S.close()
