"""GPU parity of pe_eval_jac against the oracle (needs an MI355X).

Bars: complex double-double within 1e-28 and complex FP64 within 1e-13 in
the condition-scaled metric (|y_gpu - y_oracle| / S(y), S = sum of term
magnitudes); structural zeros of the Jacobian exactly zero.
"""
import numpy as np
import pytest

import synth
from oracle import ddoracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1201_0499_amd as pe  # noqa: E402
from gpu_helpers import run_eval, scaled_err  # noqa: E402

DD_TOL = 1e-28
F64_TOL = 1e-13


def _check_dd(sys_np, pts, schedule=None, polys=None, tag=""):
    print(f"[case] dd {tag} n={sys_np.n_vars} polys={sys_np.n_polys} M={sys_np.n_monos} "
          f"P={pts[0].shape[0]} schedule={schedule}", flush=True)
    S = pe.System.from_csr(sys_np)
    if schedule:
        S.set_schedule(**schedule)
    f, J = run_eval(S, pts, pe.PE_DD)
    rf, rJ = O.eval_dd(sys_np, pts, polys=polys)
    Sf, SJ = O.scales(sys_np, pts[0], pts[2], polys=polys)
    if polys is not None:
        sel = np.asarray(polys)
        f = tuple(a[:, sel] for a in f)
        J = tuple(a[:, :, sel] for a in J)
        rf = tuple(a[:, sel] for a in rf)
        rJ = tuple(a[:, :, sel] for a in rJ)
        Sf, SJ = Sf[:, sel], SJ[:, :, sel]
    ef, zf = scaled_err(f, rf, Sf)
    eJ, zJ = scaled_err(J, rJ, SJ)
    used = S.get_schedule(pts[0].shape[0])
    S.close()
    print(f"[err] dd {tag}: max scaled error f {ef:.3e}, J {eJ:.3e} (bar {DD_TOL:.0e}), "
          f"schedule {used}", flush=True)
    assert zJ, "structural zeros of J must be exactly zero"
    assert ef < DD_TOL and eJ < DD_TOL, (ef, eJ)
    return ef, eJ


def _check_f64(sys_np, pts, schedule=None, polys=None, tag=""):
    print(f"[case] f64 {tag} n={sys_np.n_vars} M={sys_np.n_monos} P={pts[0].shape[0]} "
          f"schedule={schedule}", flush=True)
    S = pe.System.from_csr(sys_np)
    if schedule:
        S.set_schedule(**schedule)
    f, J = run_eval(S, pts, pe.PE_FP64)
    (fr, fi), (Jr, Ji) = O.eval_f64(sys_np, pts[0], pts[2], polys=polys)
    Sf, SJ = O.scales(sys_np, pts[0], pts[2], polys=polys)
    if polys is not None:
        sel = np.asarray(polys)
        f = tuple(a[:, sel] for a in f)
        J = tuple(a[:, :, sel] for a in J)
        fr, fi = fr[:, sel], fi[:, sel]
        Jr, Ji = Jr[:, :, sel], Ji[:, :, sel]
        Sf, SJ = Sf[:, sel], SJ[:, :, sel]
    ef, _ = scaled_err((f[0], f[2]), (fr, fi), Sf)
    eJ, zJ = scaled_err((J[0], J[2]), (Jr, Ji), SJ)
    used = S.get_schedule(pts[0].shape[0])
    S.close()
    print(f"[err] f64 {tag}: max scaled error f {ef:.3e}, J {eJ:.3e} (bar {F64_TOL:.0e}), "
          f"schedule {used}", flush=True)
    assert zJ
    assert ef < F64_TOL and eJ < F64_TOL, (ef, eJ)
    return ef, eJ


def test_tiny_workload_dd():
    sys_np, pts = synth.tiny_workload()
    ef, eJ = _check_dd(sys_np, pts, tag="tiny")
    assert ef < 1e-30 and eJ < 1e-30


def test_tiny_workload_fp64():
    sys_np, pts = synth.tiny_workload()
    _check_f64(sys_np, pts, tag="tiny")


@pytest.mark.parametrize("sched", [
    dict(lanes=1, chunk_vars=4, threads=64, groups=1),
    dict(lanes=2, chunk_vars=2, threads=128, groups=1),
    dict(lanes=4, chunk_vars=2, threads=256, groups=1),
    dict(lanes=1, chunk_vars=8, threads=64, groups=2),
    dict(lanes=2, chunk_vars=4, threads=64, groups=3),
])
def test_ragged_multi_chunk_schedules(sched):
    # m = 37 monomials per polynomial: several chunks plus a ragged tail
    sys_np = synth.regular_system(20, 37, 4, (1, 3), seed=7, n_polys=11)
    pts = synth.points(3, 20, 8)
    _check_dd(sys_np, pts, schedule=sched, tag="ragged")
    _check_f64(sys_np, pts, schedule=sched, tag="ragged")


def test_special_cases_dd():
    """k = 0 constants, k = 1, a zero coefficient, a duplicated monomial, an
    empty polynomial, high exponents, non-square shape."""
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
    coefs[0][1] = (0.0, 0.0, 0.0, 0.0)
    sys_np = synth.system_from_lists(5, polys, coefs)
    pts = synth.points(4, 5, 55)
    _check_dd(sys_np, pts, tag="special")
    _check_f64(sys_np, pts, tag="special")


@pytest.mark.parametrize("sched", [
    None,
    dict(lanes=2, chunk_vars=2, threads=64, groups=1),
    dict(lanes=2, chunk_vars=2, threads=128, groups=2),
    dict(lanes=1, chunk_vars=4, threads=64, groups=3),
])
def test_constant_monomials(sched):
    """A constant last in its polynomial starts the value output's
    accumulator instead of taking a chunk slot: a polynomial that is only a
    constant, two trailing constants, a leading constant, and a trailing one
    after several chunks, under single and split workgroups."""
    polys = [[[]], [[(0, 1)], [], []], [[], [(1, 2), (2, 1)]], [[(0, 1), (2, 3)], []]]
    rng = synth.rng_for(77)
    coefs = []
    for monos in polys:
        pl = synth.unit_circle_dd(rng, (len(monos),))
        coefs.append([tuple(float(a[j]) for a in pl) for j in range(len(monos))])
    small = synth.system_from_lists(3, polys, coefs)
    pts = synth.points(3, 3, 78)
    _check_dd(small, pts, schedule=sched, tag="constants")
    _check_f64(small, pts, schedule=sched, tag="constants")
    # 130 monomials + a constant per polynomial: three chunks of 64 lanes
    kr, _ = synth.known_root_system(12, 130, 3, (1, 3), seed=79)
    pts = synth.points(2, 12, 80)
    _check_dd(kr, pts, schedule=sched, tag="known-root")
    _check_f64(kr, pts, schedule=sched, tag="known-root")


@pytest.mark.parametrize("sched", [
    dict(lanes=2, chunk_vars=4, threads=64, groups=1),
    dict(lanes=1, chunk_vars=8, threads=128, groups=2),
])
def test_many_summation_rounds(sched):
    """n = 300: 301 outputs on 64 or 128 lanes, so the summation takes three
    to five rounds of ranks, alternating in direction (the first three
    requested ahead, the rest in the loop)."""
    sys_np = synth.regular_system(300, 40, 8, (1, 3), seed=17, n_polys=4)
    pts = synth.points(2, 300, 18)
    _check_dd(sys_np, pts, schedule=sched, tag="rounds")
    _check_f64(sys_np, pts, schedule=sched, tag="rounds")


@pytest.mark.parametrize("sched", [None, dict(lanes=4, chunk_vars=4, threads=512, groups=2)],
                         ids=["auto", "lanes4_cv4_t512_g2"])
def test_paper_scale_full_dd_all_rows(sched):
    """n=128, m=256, k=16, exponents 1..3, one point: every output (all 128
    values and all 128 x 128 Jacobian entries) against the oracle, in the
    automatic schedule and in the split schedule the single-point
    measurement runs (two workgroups per polynomial plus the combine)."""
    sys_np, pts = synth.paper_scale_workload()
    _check_dd(sys_np, pts, schedule=sched, tag="paper_scale all rows")


def test_paper_scale_fp64_full():
    sys_np, pts = synth.paper_scale_workload()
    _check_f64(sys_np, pts, tag="paper_scale")


def test_large_shape_dd_sampled():
    """n=512, m=1024, k=32, exponents 1..5 at 2 points; 3 polynomials checked."""
    sys_np = synth.regular_system(512, 1024, 32, (1, 5), seed=synth.config_seed(4))
    pts = synth.points(2, 512, synth.config_seed(4) + 1)
    _check_dd(sys_np, pts, polys=[0, 255, 511], tag="large")


def test_large_shape_fp64_sampled():
    """The large workload in complex FP64 (n=512, m=1024, k=32, exponents
    1..5) at 2 points, in the schedule the 256-point launch uses (eight
    lanes of four variables per monomial, 512 threads); all outputs of 3
    polynomials against the oracle."""
    sys_np = synth.regular_system(512, 1024, 32, (1, 5), seed=synth.config_seed(4))
    pts = synth.points(2, 512, synth.config_seed(4) + 1)
    S = pe.System.from_csr(sys_np)
    big = S.get_schedule(256)
    S.close()
    assert {k: big[k] for k in ("lanes", "chunk_vars", "threads", "groups")} == \
        dict(lanes=8, chunk_vars=4, threads=512, groups=1), big
    _check_f64(sys_np, pts, schedule=big, polys=[0, 255, 511], tag="large")


def test_batch_like_systems_dd():
    """Uneven shapes like the batched workload (n, m, k drawn at random)."""
    systems, pts = synth.batch_workload(n_systems=5, points_per_system=3)
    for s, p in zip(systems, pts):
        sel = sorted({0, s.n_polys // 2, s.n_polys - 1})
        _check_dd(s, p, polys=sel, tag=f"batchlike k={s.max_k}")


def test_determinism_bitwise():
    sys_np, pts = synth.paper_scale_workload()
    S = pe.System.from_csr(sys_np)
    f1, J1 = run_eval(S, pts, pe.PE_DD)
    f2, J2 = run_eval(S, pts, pe.PE_DD)
    for a, b in zip(f1 + J1, f2 + J2):
        assert np.array_equal(a, b)
    S.close()


@pytest.mark.parametrize("sched", [
    dict(lanes=4, chunk_vars=4, threads=512, groups=2),
    dict(lanes=4, chunk_vars=4, threads=256, groups=4),
])
def test_split_polynomials_paper_scale(sched):
    """Polynomials split over 2 and 4 workgroups, whose partial rows are
    added afterwards: paper-scale system at 4 points, all outputs of 6
    polynomials against the oracle, then two more launches that must repeat
    the first bit for bit."""
    sys_np, _ = synth.paper_scale_workload()
    pts = synth.points(4, sys_np.n_vars, 91)
    _check_dd(sys_np, pts, schedule=sched, polys=[0, 1, 37, 64, 100, 127], tag="split")
    S = pe.System.from_csr(sys_np)
    S.set_schedule(**sched)
    f1, J1 = run_eval(S, pts, pe.PE_DD)
    f2, J2 = run_eval(S, pts, pe.PE_DD)
    for a, b in zip(f1 + J1, f2 + J2):
        assert np.array_equal(a, b)
    S.close()


def test_values_only_and_zero_points():
    sys_np, pts = synth.tiny_workload()
    S = pe.System.from_csr(sys_np)
    f, J = run_eval(S, pts, pe.PE_DD, with_jac=False)
    rf, _ = O.eval_dd(sys_np, pts, with_jac=False)
    Sf, _ = O.scales(sys_np, pts[0], pts[2], with_jac=False)
    ef, _ = scaled_err(f, rf, Sf)
    assert ef < DD_TOL and J is None
    # n_points == 0 is a no-op
    import torch as T
    z = tuple(T.zeros(1, dtype=T.float64, device="cuda") for _ in range(4))
    pe.eval_jac(S.handle, 0, z, z, None, pe.PE_DD)
    S.close()
