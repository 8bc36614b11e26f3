"""GPU parity of point tiles and double-buffered staging (needs an MI355X).

A tile of T consecutive points shares one read of each chunk's supports,
slots and coefficients; with two staging buffers the terms of the next
(chunk, point) item are computed while the previous one is summed.  Neither
changes the arithmetic or its order, so every output must equal, bit for
bit, the one-point, one-buffer launch of the same schedule, which is itself
checked against the oracle (1e-28 scaled in double-double, 1e-13 in FP64).
Point counts leave a ragged last tile.
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
from gpu_helpers import dev, host, run_eval, scaled_err  # noqa: E402

SHAPES = [(T, nbuf) for T in (1, 2, 4, 8) for nbuf in (1, 2)]


def _bitwise(a, b):
    return all(np.array_equal(u.view(np.uint64), v.view(np.uint64)) for u, v in zip(a, b))


def _oracle_check(sys_np, pts, f, J, prec, polys=None):
    Sf, SJ = O.scales(sys_np, pts[0], pts[2], polys=polys)
    sel = np.arange(sys_np.n_polys) if polys is None else np.asarray(polys)
    if prec == pe.PE_DD:
        rf, rJ = O.eval_dd(sys_np, pts, polys=polys)
        got_f, got_J = f, J
        bar = 1e-28
    else:
        (fr, fi), (Jr, Ji) = O.eval_f64(sys_np, pts[0], pts[2], polys=polys)
        rf, rJ = (fr, fi), (Jr, Ji)
        got_f, got_J = (f[0], f[2]), (J[0], J[2])
        bar = 1e-13
    ef, _ = scaled_err(tuple(a[:, sel] for a in got_f), tuple(a[:, sel] for a in rf), Sf[:, sel])
    eJ, zJ = scaled_err(tuple(a[:, :, sel] for a in got_J), tuple(a[:, :, sel] for a in rJ),
                        SJ[:, :, sel])
    return ef, eJ, zJ, bar


def _sweep(sys_np, pts, base, prec, tag, polys=None, shapes=SHAPES):
    S = pe.System.from_csr(sys_np)
    ref = None
    for T, nbuf in shapes:
        S.set_schedule(**base, tile_points=T, stage_buffers=nbuf)
        print(f"[case] tiles {tag} prec={prec} T={T} nbuf={nbuf} P={pts[0].shape[0]} "
              f"schedule={base}", flush=True)
        f, J = run_eval(S, pts, prec)
        if ref is None:
            ef, eJ, zJ, bar = _oracle_check(sys_np, pts, f, J, prec, polys)
            print(f"[err] tiles {tag} prec={prec}: f {ef:.3e}, J {eJ:.3e} (bar {bar:.0e})",
                  flush=True)
            assert zJ and ef < bar and eJ < bar
            ref = (f, J)
        else:
            assert _bitwise(f, ref[0]) and _bitwise(J, ref[1]), (T, nbuf)
    S.close()


@pytest.mark.parametrize("prec", [1, 0], ids=["dd", "fp64"])
def test_tiles_ragged_multi_chunk(prec):
    """m = 37 in chunks of 32 (two per polynomial, one ragged), 7 points."""
    sys_np = synth.regular_system(20, 37, 4, (1, 3), seed=701, n_polys=11)
    pts = synth.points(7, 20, 702)
    _sweep(sys_np, pts, dict(lanes=2, chunk_vars=2, threads=64, groups=1), prec, "ragged")


@pytest.mark.parametrize("prec", [1, 0], ids=["dd", "fp64"])
def test_tiles_split_polynomials(prec):
    """Paper-scale system split over two workgroups per polynomial (partial
    rows and the combine), 5 points; 6 polynomials against the oracle."""
    sys_np, _ = synth.paper_scale_workload()
    pts = synth.points(5, sys_np.n_vars, 703)
    _sweep(sys_np, pts, dict(lanes=4, chunk_vars=4, threads=256, groups=2), prec, "split",
           polys=[0, 1, 63, 64, 100, 127], shapes=[(1, 1), (2, 2), (4, 1), (4, 2), (8, 1)])


@pytest.mark.parametrize("prec", [1, 0], ids=["dd", "fp64"])
def test_tiles_many_summation_rounds(prec):
    """n = 300 on 64 lanes: several rounds of ranks per item, 3 points."""
    sys_np = synth.regular_system(300, 40, 8, (1, 3), seed=704, n_polys=4)
    pts = synth.points(3, 300, 705)
    _sweep(sys_np, pts, dict(lanes=2, chunk_vars=4, threads=64, groups=1), prec, "rounds",
           shapes=[(1, 1), (2, 2), (4, 2)])


def test_tiles_constants_and_newton_mask():
    """Known-root system (constant folded into the value accumulators) under
    Newton's start mask: mixed Newton with tiles of 4 points and two buffers
    follows the one-point launch bit for bit, start by start."""
    sys_np, xstar = synth.known_root_system(24, 40, 5, (1, 3), seed=706)
    starts = synth.perturbed_starts(xstar, 13, 1e-6, seed=707)
    outs = []
    for T, nbuf in ((1, 1), (4, 2), (8, 1)):
        S = pe.System.from_csr(sys_np)
        S.set_schedule(lanes=2, chunk_vars=4, threads=64, groups=1, tile_points=T,
                       stage_buffers=nbuf)
        P = starts[0].shape[0]
        x = dev(starts)
        res = torch.zeros(P, dtype=torch.float64, device="cuda")
        it = torch.zeros(P, dtype=torch.int32, device="cuda")
        st = torch.zeros(P, dtype=torch.int32, device="cuda")
        code = S.newton(P, x, res, it, st, tol=1e-28, max_iter=10, mode=pe.PE_NEWTON_MIXED)
        torch.cuda.synchronize()
        outs.append((host(x), it.cpu().numpy(), st.cpu().numpy()))
        S.close()
        print(f"[case] tiles newton T={T} nbuf={nbuf}: code {code}, iterations "
              f"{np.bincount(outs[-1][1]).tolist()}", flush=True)
        assert code == 0 and np.all(outs[-1][2] == 0)
    for x, it, st in outs[1:]:
        assert _bitwise(x, outs[0][0]) and np.array_equal(it, outs[0][1])


@pytest.mark.parametrize("prec", [1, 0], ids=["dd", "fp64"])
def test_tiles_large_shape(prec):
    """n=512, m=1024, k=32, exponents 1..5, 256 threads: what fits the LDS
    (one point with two buffers in dd; two points with one or two buffers in
    FP64), 3 points, 3 polynomials against the oracle and every output
    against the one-point launch."""
    sys_np = synth.regular_system(512, 1024, 32, (1, 5), seed=synth.config_seed(4))
    pts = synth.points(3, 512, synth.config_seed(4) + 2)
    base = dict(lanes=8, chunk_vars=4, threads=256, groups=1)
    shapes = [(1, 1), (1, 2)] if prec == pe.PE_DD else [(1, 1), (2, 1), (2, 2)]
    _sweep(sys_np, pts, base, prec, "large", polys=[0, 255, 511], shapes=shapes)


def test_tile_that_does_not_fit_is_refused():
    sys_np = synth.regular_system(512, 64, 32, (1, 5), seed=708, n_polys=2)
    S = pe.System.from_csr(sys_np)
    S.set_schedule(lanes=8, chunk_vars=4, threads=256, groups=1, tile_points=8, stage_buffers=2)
    pts = synth.points(8, 512, 709)
    with pytest.raises(pe.PolyevalError) as ei:
        run_eval(S, pts, pe.PE_DD)
    assert ei.value.status == 4 and "LDS" in str(ei.value)
    S.close()
