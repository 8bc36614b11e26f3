"""GPU parity of pe_eval_jac_paper_layout (the paper's three-kernel
evaluation: common factors, monomial terms into the dense zero-padded term
array, one thread per output) against the oracle, with the same bars as
pe_eval_jac: complex double-double within 1e-28 and complex FP64 within
1e-13 in the condition-scaled metric, structural zeros exactly zero."""
import numpy as np
import pytest

import synth
from oracle import ddoracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1201_0499_amd as pe  # noqa: E402
from gpu_helpers import alloc, dev, host, scaled_err  # noqa: E402


def _run(S, sys_np, pts, precision):
    P = pts[0].shape[0]
    f = alloc((P, sys_np.n_polys))
    J = alloc((P, sys_np.n_vars, sys_np.n_polys))
    S.eval_jac_paper_layout(P, dev(pts), f, J, precision)
    torch.cuda.synchronize()
    return host(f), host(J)


def _check(S, sys_np, pts, polys=None, tag=""):
    print(f"[case] paper layout {tag} n={sys_np.n_vars} M={sys_np.n_monos} P={pts[0].shape[0]}",
          flush=True)
    f, J = _run(S, sys_np, pts, pe.PE_DD)
    rf, rJ = O.eval_dd(sys_np, pts, polys=polys)
    Sf, SJ = O.scales(sys_np, pts[0], pts[2], polys=polys)
    if polys is not None:
        sel = np.asarray(polys)
        f = tuple(a[:, sel] for a in f)
        J = tuple(a[:, :, sel] for a in J)
        rf = tuple(a[:, sel] for a in rf)
        rJ = tuple(a[:, :, sel] for a in rJ)
        Sf, SJ = Sf[:, sel], SJ[:, :, sel]
    ef, _ = scaled_err(f, rf, Sf)
    eJ, zJ = scaled_err(J, rJ, SJ)
    assert zJ and ef < 1e-28 and eJ < 1e-28, (ef, eJ)
    f, J = _run(S, sys_np, pts, pe.PE_FP64)
    (fr, fi), (Jr, Ji) = O.eval_f64(sys_np, pts[0], pts[2])
    Sf, SJ = O.scales(sys_np, pts[0], pts[2])
    if polys is not None:
        sel = np.asarray(polys)
        f = tuple(a[:, sel] for a in f)
        J = tuple(a[:, :, sel] for a in J)
        fr, fi, Jr, Ji = fr[:, sel], fi[:, sel], Jr[:, :, sel], Ji[:, :, sel]
        Sf, SJ = Sf[:, sel], SJ[:, :, sel]
    ef, _ = scaled_err((f[0], f[2]), (fr, fi), Sf)
    eJ, zJ = scaled_err((J[0], J[2]), (Jr, Ji), SJ)
    assert zJ and ef < 1e-13 and eJ < 1e-13, (ef, eJ)


def test_tiny_and_ragged():
    sys_np, pts = synth.tiny_workload()
    S = pe.System.from_csr(sys_np)
    _check(S, sys_np, pts, tag="tiny")
    S.close()
    sys_np = synth.regular_system(20, 37, 4, (1, 3), seed=7, n_polys=11)
    S = pe.System.from_csr(sys_np)
    # point counts and precisions alternate, so the dense array is laid out again
    _check(S, sys_np, synth.points(3, 20, 8), tag="ragged P=3")
    _check(S, sys_np, synth.points(2, 20, 9), tag="ragged P=2")
    S.close()


def test_special_cases():
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
    S = pe.System.from_csr(sys_np)
    _check(S, sys_np, synth.points(4, 5, 55), tag="special")
    S.close()


def test_paper_scale_sampled():
    sys_np, pts = synth.paper_scale_workload()
    S = pe.System.from_csr(sys_np)
    _check(S, sys_np, pts, polys=[0, 37, 127], tag="paper scale")
    S.close()
