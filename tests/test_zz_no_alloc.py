"""GPU test of pe_eval_jac_noalloc, the allocation-free variant of
pe_eval_jac, called through the C interface.

It runs the same kernels as pe_eval_jac under the same schedule, with the
partial rows of a split polynomial (groups > 1) in the library's static
device scratch, so its outputs must equal pe_eval_jac's bit for bit.  Two
calls in a row, the second on fewer points, each checked against
pe_eval_jac; the outputs are also checked against the oracle on a few rows.
"""
import ctypes as C

import numpy as np
import pytest

import synth
from oracle import ddoracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1201_0499_amd as pe  # noqa: E402
from paper_1201_0499_amd import _abi  # noqa: E402
from gpu_helpers import alloc, dev, host, scaled_err  # noqa: E402

PE_EUNSUPPORTED = 4
SCRATCH_BYTES = 32 << 20


def _planes(ts):
    return _abi.cvec([t.data_ptr() if t is not None else 0 for t in ts])


def _call(fn, S, P, x, f, J, prec):
    stream = torch.cuda.current_stream().cuda_stream
    return fn(C.c_void_p(S.handle), P, _planes(x), _planes(f), _planes(J), prec,
              C.c_void_p(stream))


def _bitwise_equal(a, b):
    return all(np.array_equal(u.view(np.uint64), v.view(np.uint64)) for u, v in zip(a, b))


def _case(S, sys_np, pts, prec, tag):
    L = pe.lib()
    P = pts[0].shape[0]
    n, npoly = sys_np.n_vars, sys_np.n_polys
    nplanes = 4
    x = dev(pts)
    f_ref, J_ref = alloc((P, npoly), nplanes), alloc((P, n, npoly), nplanes)
    f_na, J_na = alloc((P, npoly), nplanes), alloc((P, n, npoly), nplanes)
    print(f"[case] noalloc {tag} n={n} polys={npoly} P={P} prec={prec} "
          f"schedule={S.get_schedule(P)}", flush=True)
    assert _call(L.pe_eval_jac, S, P, x, f_ref, J_ref, prec) == 0, L.pe_last_error()
    st = _call(L.pe_eval_jac_noalloc, S, P, x, f_na, J_na, prec)
    assert st == 0, L.pe_last_error()
    torch.cuda.synchronize()
    fr, Jr, fn, Jn = host(f_ref), host(J_ref), host(f_na), host(J_na)
    if prec == pe.PE_FP64:
        fr, Jr, fn, Jn = ((a[0], a[2]) for a in (fr, Jr, fn, Jn))
    assert _bitwise_equal(fn, fr) and _bitwise_equal(Jn, Jr), f"{tag}: differs from pe_eval_jac"
    # a few rows against the oracle as well
    polys = [0, npoly // 2, npoly - 1]
    Sf, SJ = O.scales(sys_np, pts[0], pts[2], polys=polys)
    sel = np.asarray(polys)
    if prec == pe.PE_DD:
        rf, rJ = O.eval_dd(sys_np, pts, polys=polys)
        ef, _ = scaled_err(tuple(a[:, sel] for a in fn), tuple(a[:, sel] for a in rf), Sf[:, sel])
        eJ, zJ = scaled_err(tuple(a[:, :, sel] for a in Jn), tuple(a[:, :, sel] for a in rJ),
                            SJ[:, :, sel])
        bar = 1e-28
    else:
        (rfr, rfi), (rJr, rJi) = O.eval_f64(sys_np, pts[0], pts[2], polys=polys)
        ef, _ = scaled_err(tuple(a[:, sel] for a in fn), (rfr[:, sel], rfi[:, sel]), Sf[:, sel])
        eJ, zJ = scaled_err(tuple(a[:, :, sel] for a in Jn), (rJr[:, :, sel], rJi[:, :, sel]),
                            SJ[:, :, sel])
        bar = 1e-13
    print(f"[err] noalloc {tag}: bitwise equal to pe_eval_jac; oracle rows {polys}: "
          f"f {ef:.3e}, J {eJ:.3e} (bar {bar:.0e})", flush=True)
    assert zJ and ef < bar and eJ < bar


@pytest.mark.parametrize("prec", [1, 0], ids=["dd", "fp64"])
def test_noalloc_split_schedule_two_calls(prec):
    """Paper-scale system with each polynomial split over two workgroups (the
    partial rows go through the static scratch): 3 points, then 1."""
    sys_np, _ = synth.paper_scale_workload()
    S = pe.System.from_csr(sys_np)
    S.set_schedule(lanes=4, chunk_vars=4, threads=512, groups=2)
    for P, seed in ((3, 77), (1, 78)):
        pts = synth.points(P, sys_np.n_vars, seed)
        _case(S, sys_np, pts, prec, f"paper-scale groups=2 P={P}")
    S.close()


def test_noalloc_automatic_schedule_two_calls():
    """A smaller system under its automatic schedule: 5 points, then 2."""
    sys_np = synth.regular_system(24, 40, 6, exp_range=(1, 3), seed=1201)
    S = pe.System.from_csr(sys_np)
    for P, seed in ((5, 91), (2, 92)):
        pts = synth.points(P, sys_np.n_vars, seed)
        _case(S, sys_np, pts, pe.PE_DD, f"regular n=24 P={P}")
    S.close()


def test_noalloc_rejections():
    """Without prepared tables, and above the scratch size, the call fails
    before launching anything."""
    L = pe.lib()
    sys_np, _ = synth.paper_scale_workload()
    n, npoly = sys_np.n_vars, sys_np.n_polys
    S = pe.System.from_csr(sys_np)
    S.set_schedule(lanes=4, chunk_vars=4, threads=512, groups=2)
    per_point = 2 * npoly * (n + 1) * 32          # partial rows of one point in dd
    P = SCRATCH_BYTES // per_point + 1            # one point more than fits
    assert P * per_point > SCRATCH_BYTES
    pts = synth.points(P, n, 5)
    x = dev(pts)
    f, J = alloc((P, npoly)), alloc((P, n, npoly))
    st = _call(L.pe_eval_jac_noalloc, S, P, x, f, J, pe.PE_DD)
    assert st == PE_EUNSUPPORTED and b"pe_eval_jac once" in L.pe_last_error()
    # prepare the (pinned) schedule's tables with a small call, then ask for too many points
    assert _call(L.pe_eval_jac, S, 1, x, f, J, pe.PE_DD) == 0
    st = _call(L.pe_eval_jac_noalloc, S, P, x, f, J, pe.PE_DD)
    assert st == PE_EUNSUPPORTED and b"static scratch" in L.pe_last_error()
    print(f"[err] noalloc rejections: {L.pe_last_error().decode()}", flush=True)
    # in FP64 the same points fit (16 bytes per value): the call succeeds
    st = _call(L.pe_eval_jac_noalloc, S, P, x, f, J, pe.PE_FP64)
    assert st == 0, L.pe_last_error()
    torch.cuda.synchronize()
    S.close()
