"""GPU parity at the exact configurations bench.py times (needs an MI355X).

bench.py takes its launch schedules from the autotuners with the committed
cache paper_1201_0499_amd/tuned_schedules.txt.  These tests ask the same
autotuners with the same cache and the same workload shapes, so they run
the schedules the measurements run, at full size, and check sampled outputs
against the oracle (1e-28 scaled in double-double, 1e-13 in FP64): the
large system at all 256 points (two points, three polynomials checked), the
paper-scale system at one point (every output), and the batch of 64 uneven
systems at 64 points each (two points and three polynomials of every
system).
"""
import os

import numpy as np
import pytest

import synth
from oracle import ddoracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1201_0499_amd as pe  # noqa: E402
from gpu_helpers import dev, scaled_err  # noqa: E402
from tuned_keys import TUNED, bench_system_keys, read_tuned  # noqa: E402


def _alloc(P, npoly, n):
    f = tuple(torch.full((P, npoly), float("nan"), dtype=torch.float64, device="cuda")
              for _ in range(4))
    J = tuple(torch.full((P, n, npoly), float("nan"), dtype=torch.float64, device="cuda")
              for _ in range(4))
    return f, J


def _check(sys_np, pts, f, J, prec, pts_sel, polys, tag):
    """Oracle check of points pts_sel and polynomials polys of device outputs."""
    sub = tuple(a[pts_sel] for a in pts)
    fs = tuple(t[pts_sel].cpu().numpy() for t in f)
    Js = tuple(t[pts_sel].cpu().numpy() for t in J)
    sel = np.asarray(polys)
    Sf, SJ = O.scales(sys_np, sub[0], sub[2], polys=polys)
    if prec == pe.PE_DD:
        rf, rJ = O.eval_dd(sys_np, sub, polys=polys)
        ef, _ = scaled_err(tuple(a[:, sel] for a in fs), tuple(a[:, sel] for a in rf), Sf[:, sel])
        eJ, zJ = scaled_err(tuple(a[:, :, sel] for a in Js), tuple(a[:, :, sel] for a in rJ),
                            SJ[:, :, sel])
        bar = 1e-28
    else:
        (fr, fi), (Jr, Ji) = O.eval_f64(sys_np, sub[0], sub[2], polys=polys)
        ef, _ = scaled_err((fs[0][:, sel], fs[2][:, sel]), (fr[:, sel], fi[:, sel]), Sf[:, sel])
        eJ, zJ = scaled_err((Js[0][:, :, sel], Js[2][:, :, sel]), (Jr[:, :, sel], Ji[:, :, sel]),
                            SJ[:, :, sel])
        bar = 1e-13
    print(f"[err] bench config {tag}: max scaled error f {ef:.3e}, J {eJ:.3e} (bar {bar:.0e})",
          flush=True)
    assert zJ and ef < bar and eJ < bar


def _system_case(sys_np, pts, prec, key, pts_sel, polys, tag):
    tuned = read_tuned()
    assert key in tuned, f"{key} missing from {TUNED}"
    P = pts[0].shape[0]
    S = pe.System.from_csr(sys_np)
    x = dev(pts)
    f, J = _alloc(P, sys_np.n_polys, sys_np.n_vars)
    S.autotune(P, x, f, J, prec, cache_path=TUNED)
    sched = S.get_schedule(P)
    want = dict(zip(("lanes", "chunk_vars", "threads", "groups", "tile_points",
                     "stage_buffers"), tuned[key]))
    print(f"[case] bench config {tag}: schedule {sched}", flush=True)
    assert sched == want, (sched, want)
    S.eval_jac(P, x, f, J, prec)
    torch.cuda.synchronize()
    _check(sys_np, pts, f, J, prec, pts_sel, polys, tag)
    S.close()


@pytest.mark.parametrize("prec", [1, 0], ids=["dd", "fp64"])
def test_large_workload_at_bench_schedule(prec):
    """n=512, m=1024, k=32, exponents 1..5, all 256 points in one launch."""
    sys_np, pts = synth.large_workload()
    key = bench_system_keys()[("large", prec)]
    _system_case(sys_np, pts, prec, key, [0, 255], [0, 255, 511], f"large prec={prec}")


@pytest.mark.parametrize("prec", [1, 0], ids=["dd", "fp64"])
def test_paper_scale_at_bench_schedule(prec):
    """n=128, m=256, k=16, exponents 1..3, one point: every output."""
    sys_np, pts = synth.paper_scale_workload()
    key = bench_system_keys()[("paper_scale", prec)]
    _system_case(sys_np, pts, prec, key, [0], list(range(sys_np.n_polys)),
                 f"paper-scale prec={prec}")


def test_batch_at_bench_config():
    """64 uneven systems at 64 points each, one launch, the tuned batch
    configuration: points 0 and 63 of every system, three polynomials."""
    systems, pts = synth.batch_workload()
    S = [pe.System.from_csr(s) for s in systems]
    B = pe.Batch(S)
    pps = np.array([p[0].shape[0] for p in pts], np.int64)
    xo, fo, jo = B.layout(pps)
    x = tuple(torch.from_numpy(np.concatenate([p[q].reshape(-1) for p in pts])).cuda()
              for q in range(4))
    f = tuple(torch.full((int(fo[-1]),), float("nan"), dtype=torch.float64, device="cuda")
              for _ in range(4))
    J = tuple(torch.full((int(jo[-1]),), float("nan"), dtype=torch.float64, device="cuda")
              for _ in range(4))
    assert os.path.exists(TUNED)
    B.autotune(pps, x, f, J, pe.PE_DD, cache_path=TUNED)
    print(f"[case] bench config batch: {B.config()}", flush=True)
    B.eval_jac(pps, x, f, J, pe.PE_DD)
    torch.cuda.synchronize()
    worst_f = worst_J = 0.0
    for i, (s, p) in enumerate(zip(systems, pts)):
        P = p[0].shape[0]
        sel_pts = [0, P - 1]
        fb = tuple(t[int(fo[i]):int(fo[i + 1])].view(P, s.n_polys)[sel_pts].cpu().numpy() for t in f)
        Jb = tuple(t[int(jo[i]):int(jo[i + 1])].view(P, s.n_vars, s.n_polys)[sel_pts].cpu().numpy()
                   for t in J)
        sub = tuple(a[sel_pts] for a in p)
        polys = sorted({0, s.n_polys // 2, s.n_polys - 1})
        sel = np.asarray(polys)
        rf, rJ = O.eval_dd(s, sub, polys=polys)
        Sf, SJ = O.scales(s, sub[0], sub[2], polys=polys)
        ef, _ = scaled_err(tuple(a[:, sel] for a in fb), tuple(a[:, sel] for a in rf), Sf[:, sel])
        eJ, z = scaled_err(tuple(a[:, :, sel] for a in Jb), tuple(a[:, :, sel] for a in rJ),
                           SJ[:, :, sel])
        assert z, f"system {i}: structural zeros"
        worst_f, worst_J = max(worst_f, ef), max(worst_J, eJ)
    print(f"[err] bench config batch: max scaled error f {worst_f:.3e}, J {worst_J:.3e} "
          f"(bar 1e-28)", flush=True)
    assert worst_f < 1e-28 and worst_J < 1e-28
    B.close()
    for s in S:
        s.close()
