"""Batched persistent launch (pe_eval_jac_batch): parity with the per-system
path and the oracle, hipGraph capture and replay, and the autotuner."""
import os
import tempfile

import numpy as np
import pytest

import synth
from oracle import ddoracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1201_0499_amd as pe  # noqa: E402
from gpu_helpers import dev, host, scaled_err  # noqa: E402


def _concat(planes_list):
    return tuple(np.concatenate([p[q].reshape(-1) for p in planes_list]) for q in range(4))


def _setup(n_systems=6, pts_per=3, seed_rep=1):
    systems, pts = synth.batch_workload(n_systems=n_systems, points_per_system=pts_per,
                                        replicate=seed_rep)
    S = [pe.System.from_csr(s) for s in systems]
    B = pe.Batch(S)
    pps = np.array([p[0].shape[0] for p in pts], np.int64)
    xo, fo, jo = B.layout(pps)
    x = dev(_concat(pts))
    f = tuple(torch.full((int(fo[-1]),), float("nan"), dtype=torch.float64, device="cuda") for _ in range(4))
    J = tuple(torch.full((int(jo[-1]),), float("nan"), dtype=torch.float64, device="cuda") for _ in range(4))
    return systems, pts, S, B, pps, (xo, fo, jo), x, f, J


def _block(planes, off, i, shape):
    return tuple(a[off[i]:off[i + 1]].reshape(shape) for a in planes)


@pytest.mark.parametrize("prec", [1, 0], ids=["dd", "fp64"])
def test_batch_matches_single_system_bitwise_and_oracle(prec):
    systems, pts, S, B, pps, (xo, fo, jo), x, f, J = _setup()
    print(f"[case] batch prec={prec} shapes={[(s.n_vars, s.n_monos, s.max_k) for s in systems]}", flush=True)
    B.eval_jac(pps, x, f, J, prec)
    torch.cuda.synchronize()
    fh, Jh = host(f), host(J)
    cfg = B.config()
    for i, (s, p) in enumerate(zip(systems, pts)):
        P = p[0].shape[0]
        fb = _block(fh, fo, i, (P, s.n_polys))
        Jb = _block(Jh, jo, i, (P, s.n_vars, s.n_polys))
        # same schedule through the single-system entry point: identical bits
        L = min(32, (1 << max(0, int(np.ceil(np.log2(max(1, -(-s.max_k // cfg["chunk_vars"])))))))
                * cfg["lanes_mult"])
        S[i].set_schedule(L, cfg["chunk_vars"], cfg["threads"], 1)
        x1 = dev(p)
        f1 = tuple(torch.empty((P, s.n_polys), dtype=torch.float64, device="cuda") for _ in range(4))
        J1 = tuple(torch.empty((P, s.n_vars, s.n_polys), dtype=torch.float64, device="cuda") for _ in range(4))
        S[i].eval_jac(P, x1, f1, J1, prec)
        torch.cuda.synchronize()
        planes = (0, 1, 2, 3) if prec == 1 else (0, 2)
        for q in planes:
            assert np.array_equal(fb[q], f1[q].cpu().numpy())
            assert np.array_equal(Jb[q], J1[q].cpu().numpy())
        # oracle on three polynomials
        sel = sorted({0, s.n_polys // 2, s.n_polys - 1})
        if prec == 1:
            rf, rJ = O.eval_dd(s, p, polys=sel)
            Sf, SJ = O.scales(s, p[0], p[2], polys=sel)
            ef, _ = scaled_err(tuple(a[:, sel] for a in fb), tuple(a[:, sel] for a in rf), Sf[:, sel])
            eJ, z = scaled_err(tuple(a[:, :, sel] for a in Jb), tuple(a[:, :, sel] for a in rJ), SJ[:, :, sel])
            assert z and ef < 1e-28 and eJ < 1e-28
        else:
            (rfr, rfi), (rJr, rJi) = O.eval_f64(s, p[0], p[2])
            Sf, SJ = O.scales(s, p[0], p[2])
            ef, _ = scaled_err((fb[0], fb[2]), (rfr, rfi), Sf)
            eJ, z = scaled_err((Jb[0], Jb[2]), (rJr, rJi), SJ)
            assert z and ef < 1e-13 and eJ < 1e-13
    B.close()
    for s in S:
        s.close()


def test_batch_graph_capture_replays_match_eager():
    systems, pts, S, B, pps, lay, x, f, J = _setup(n_systems=5, pts_per=2, seed_rep=2)
    B.eval_jac(pps, x, f, J, 1)           # builds the task list outside capture
    torch.cuda.synchronize()
    ref = [t.clone() for t in f + J]
    st = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        B.eval_jac(pps, x, f, J, 1, stream=st)
    for rep in range(3):
        for t in f + J:
            t.fill_(float("nan"))          # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(f + J, ref):
            assert torch.equal(a, b), f"replay {rep} differs"
    B.close()
    for s in S:
        s.close()


def test_autotune_batch_and_cache():
    systems, pts, S, B, pps, lay, x, f, J = _setup(n_systems=4, pts_per=2, seed_rep=3)
    path = os.path.join(tempfile.mkdtemp(), "tune.txt")
    B.autotune(pps, x, f, J, 1, cache_path=path)
    cfg = B.config()
    assert cfg["chunk_vars"] in (2, 4, 8) and cfg["threads"] in (256, 512)
    assert os.path.exists(path) and open(path).read().strip()
    # results after tuning are still right
    B.eval_jac(pps, x, f, J, 1)
    torch.cuda.synchronize()
    fh = host(f)
    xo, fo, jo = lay
    s, p = systems[0], pts[0]
    rf, _ = O.eval_dd(s, p, with_jac=False)
    Sf, _ = O.scales(s, p[0], p[2], with_jac=False)
    ef, _ = scaled_err(_block(fh, fo, 0, (p[0].shape[0], s.n_polys)), rf, Sf)
    assert ef < 1e-28
    # a new batch over the same shapes reads the cache
    B2 = pe.Batch(S)
    B2.autotune(pps, x, f, J, 1, cache_path=path)
    assert B2.config() == cfg
    B.close()
    B2.close()
    for s_ in S:
        s_.close()


def test_autotune_system_pins_a_valid_schedule():
    s, p = synth.paper_scale_workload()
    S = pe.System.from_csr(s)
    x = dev(p)
    f = tuple(torch.empty((1, s.n_polys), dtype=torch.float64, device="cuda") for _ in range(4))
    J = tuple(torch.empty((1, s.n_vars, s.n_polys), dtype=torch.float64, device="cuda") for _ in range(4))
    S.autotune(1, x, f, J, 1)
    sch = S.get_schedule(1)
    assert sch["lanes"] * sch["chunk_vars"] >= s.max_k
    S.eval_jac(1, x, f, J, 1)
    torch.cuda.synchronize()
    sel = [0, 64, 127]
    rf, rJ = O.eval_dd(s, p, polys=sel)
    Sf, SJ = O.scales(s, p[0], p[2], polys=sel)
    ef, _ = scaled_err(tuple(a.cpu().numpy()[:, sel] for a in f), tuple(a[:, sel] for a in rf), Sf[:, sel])
    assert ef < 1e-28
    S.close()


def _oracle_rows(s, p, fb, Jb, prec):
    """Max scaled errors of three polynomials (first, middle, last) of one
    system's block against the oracle."""
    sel = sorted({0, s.n_polys // 2, s.n_polys - 1})
    if prec == 1:
        rf, rJ = O.eval_dd(s, p, polys=sel)
        Sf, SJ = O.scales(s, p[0], p[2], polys=sel)
        ef, _ = scaled_err(tuple(a[:, sel] for a in fb), tuple(a[:, sel] for a in rf), Sf[:, sel])
        eJ, z = scaled_err(tuple(a[:, :, sel] for a in Jb), tuple(a[:, :, sel] for a in rJ),
                           SJ[:, :, sel])
    else:
        (rfr, rfi), (rJr, rJi) = O.eval_f64(s, p[0], p[2], polys=sel)
        Sf, SJ = O.scales(s, p[0], p[2], polys=sel)
        ef, _ = scaled_err((fb[0][:, sel], fb[2][:, sel]), (rfr[:, sel], rfi[:, sel]), Sf[:, sel])
        eJ, z = scaled_err((Jb[0][:, :, sel], Jb[2][:, :, sel]), (rJr[:, :, sel], rJi[:, :, sel]),
                           SJ[:, :, sel])
    return ef, eJ, z


@pytest.mark.parametrize("prec", [1, 0], ids=["dd", "fp64"])
def test_batch_full_workload_one_point_per_system(prec):
    """The whole batched workload (64 systems, n 16..256, m 16..1024, k
    2..16, exponents 1..4) at one point per system in one launch: three
    polynomials of every system against the oracle, first with the default
    schedule, then with the one the autotuner picks."""
    systems, pts = synth.batch_workload(n_systems=64, points_per_system=1)
    S = [pe.System.from_csr(s) for s in systems]
    B = pe.Batch(S)
    pps = np.ones(len(systems), np.int64)
    xo, fo, jo = B.layout(pps)
    x = dev(_concat(pts))
    f = tuple(torch.full((int(fo[-1]),), float("nan"), dtype=torch.float64, device="cuda") for _ in range(4))
    J = tuple(torch.full((int(jo[-1]),), float("nan"), dtype=torch.float64, device="cuda") for _ in range(4))
    for phase in ("default", "tuned"):
        if phase == "tuned":
            B.autotune(pps, x, f, J, prec)
            for t in f + J:
                t.fill_(float("nan"))
        print(f"[case] batch full prec={prec} {phase} config={B.config()}", flush=True)
        B.eval_jac(pps, x, f, J, prec)
        torch.cuda.synchronize()
        fh, Jh = host(f), host(J)
        worst_f = worst_J = 0.0
        for i, (s, p) in enumerate(zip(systems, pts)):
            fb = _block(fh, fo, i, (1, s.n_polys))
            Jb = _block(Jh, jo, i, (1, s.n_vars, s.n_polys))
            ef, eJ, z = _oracle_rows(s, p, fb, Jb, prec)
            assert z, f"system {i}: structural zeros"
            worst_f, worst_J = max(worst_f, ef), max(worst_J, eJ)
        bar = 1e-28 if prec == 1 else 1e-13
        print(f"[err] batch full prec={prec} {phase}: max scaled error f {worst_f:.3e}, "
              f"J {worst_J:.3e} (bar {bar:.0e})", flush=True)
        assert worst_f < bar and worst_J < bar
    B.close()
    for s in S:
        s.close()
