"""Throughput of the evaluation hot path on one MI355X.

Headline workload (paper-scale system): n = 128 variables, 128 polynomials
of m = 256 monomials, k = 16 variables per monomial, exponents uniform in
1..3, unit-circle complex double-double coefficients and point.  One step =
one evaluation of the system and its full Jacobian in complex double-double
at one point (one pe_eval_jac call), repeated as in Newton iterations, with the
schedule chosen by the library's autotuner (pe_autotune_system); the
launches are captured in a hipGraph of 100 launches that is replayed, so the
host does not limit the launch rate.  Inputs are resident in HBM before the
timed region.

Side measurements on the other workloads (same JSON line, "side"):
  * FP64 mode of the headline workload (its own tuned schedule);
  * Newton on a known-root system (n=128, m=256+1, k=16, exponents 1..3),
    1024 starts at 1e-6 from the root, to max|f| < 1e-28: solves/s in mixed
    precision and in all double-double;
  * a batch of 64 uneven systems (n 16..256, m 16..1024, k 2..16, exponents
    1..4, 64 points each) in one autotuned, graph-captured persistent launch;
  * the large system (n=512, m=1024, k=32, exponents 1..5) at 256 points;
  * Newton on a known-root large system (n=512, m=1024+1, k=32, exponents
    1..5), 256 starts, mixed precision and all double-double.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector (FMA counted as 2 flops)
PEAK_FP64_TINSTR = 39.3      # FP64 lane-instructions/s: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz
GRAPH_LAUNCHES = 100
COPY_BYTES = 512 << 20       # copy-calibration size


def dd_flops_per_monomial(k: int) -> int:
    """Algorithmic flops of value + all k partials of one monomial in complex
    double-double: (6k-5) complex dd products (88 flops) + (k+1) complex dd
    sums (40 flops)."""
    return 568 * k - 400


def dd_instr_per_monomial(k: int) -> int:
    """The same in FP64 instructions: 76 per product, 40 per sum."""
    return 496 * k - 340


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "eval_kernel_dd_paper_scale_traffic.json")


def kernel_sources_sha256():
    """Hash of the library sources the evaluation kernels are built from."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1201_0499_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp", ".cpp", ".h")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(sched):
    """HBM bytes per evaluation from the committed counter record (FETCH_SIZE
    and WRITE_SIZE per dispatch, each scaled by what it reads for a copy of
    known size), or None when the kernel sources or the schedule differ from
    those the counters were taken with."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("sources_sha256") != kernel_sources_sha256() or rec.get("schedule") != sched:
        return None
    return rec.get("bytes_per_evaluation")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def timed(fn, reps):
    """Milliseconds per call of fn (which enqueues GPU work), by the wall clock
    between two device synchronizations."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / reps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--skip-side", action="store_true", help="only the headline measurement")
    ap.add_argument("--no-tune", action="store_true", help="automatic schedule, no search")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1201_0499_amd", "tune_cache.txt"))
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 512 MiB (8 times), the reference for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--only", choices=["newton", "newton_large", "large", "track"],
                    help="run one side measurement alone and print its JSON (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library evaluates on one GPU: it has no collectives "
                                   "or sharding; use --gpus 1", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import synth
    import paper_1201_0499_amd as pe

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        copy_calibration(torch)
        return
    if args.only:
        stream = torch.cuda.Stream()
        run = {"newton": lambda: measure_newton(pe, torch, stream),
               "newton_large": lambda: measure_newton(pe, torch, stream, large=True),
               "large": lambda: measure_large(pe, torch, stream),
               "track": lambda: measure_track(pe, torch, stream)}[args.only]
        print(json.dumps({args.only: run()}))
        return
    dev = torch.device("cuda:0")
    sys_np, pts = synth.paper_scale_workload()
    n, npoly, M, k = sys_np.n_vars, sys_np.n_polys, sys_np.n_monos, sys_np.max_k
    log(f"[bench] workload n={n} polys={npoly} monomials={M} k={k} max_exp={sys_np.max_exp}")
    S = pe.System.from_csr(sys_np)
    x = tuple(torch.from_numpy(a).to(dev) for a in pts)
    f = tuple(torch.empty((1, npoly), dtype=torch.float64, device=dev) for _ in range(4))
    J = tuple(torch.empty((1, n, npoly), dtype=torch.float64, device=dev) for _ in range(4))
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    if not args.no_tune:
        # the library's own schedule search (timed graph replays, cached)
        S.autotune(1, x, f, J, pe.PE_DD, stream=stream, cache_path=args.tune_cache)
    sched = S.get_schedule(1)
    log(f"[bench] schedule {sched} (tuning {time.perf_counter() - t0:.1f} s)")

    def step(prec=pe.PE_DD):
        S.eval_jac(1, x, f, J, prec, stream)

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        for _ in range(GRAPH_LAUNCHES):
            step()
    with torch.cuda.stream(stream):
        graph.replay()
    torch.cuda.synchronize()
    if args.steps % GRAPH_LAUNCHES:
        args.steps += GRAPH_LAUNCHES - args.steps % GRAPH_LAUNCHES

    # ---- timed region: exactly K steps (K / 100 replays of 100 launches) ----
    # HIP events on the launch stream bracket the same region: their span / K
    # is the average time the GPU spends per evaluation (kernel plus the gap
    # to the next one inside the graph).
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(args.steps // GRAPH_LAUNCHES):
            graph.replay()
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    value = M * args.steps / wall
    kern_ms = ev0.elapsed_time(ev1) / args.steps
    log(f"[bench] dd: {ms_per_step*1e3:.2f} us/step, {value:.4e} evals/s")

    flops = M * dd_flops_per_monomial(k)
    achieved = flops / (kern_ms * 1e-3) / 1e12
    instr_rate = M * dd_instr_per_monomial(k) / (kern_ms * 1e-3) / 1e12
    log(f"[bench] dd kernel {kern_ms*1e3:.2f} us/evaluation (events), {achieved:.2f} TFLOP/s algorithmic")

    traffic = recorded_traffic(sched)
    side = {}
    if not args.skip_side:
        if not args.no_tune:
            S.autotune(1, x, f, J, pe.PE_FP64, stream=stream, cache_path=args.tune_cache)
        side.update(measure_fp64(S, step, stream, M))
        S.close()
        side["newton"] = measure_newton(pe, torch, stream)
        side["newton_large"] = measure_newton(pe, torch, stream, large=True)
        side["batch"] = measure_batch(pe, torch, stream, args.tune_cache)
        side["large"] = measure_large(pe, torch, stream)
        side["track"] = measure_track(pe, torch, stream)
        side["paper_layout"] = measure_paper_layout(pe, torch, stream, sys_np, x, f, J,
                                                    kern_ms * 1e3)
        side["quad_double"] = measure_qd(pe, torch, stream, sys_np, pts)
    else:
        S.close()

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import ddoracle as O
        reps = 0
        t0 = time.perf_counter()
        while True:
            O.eval_dd(sys_np, pts)
            reps += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds:
                break
        cpu = {"value": M * reps / el, "unit": "evals/s", "cores": 1, "kind": "oracle",
               "sample": f"{reps} full evaluations of the headline system at its point "
                         f"({reps * M} monomials with all partials) by the definitional "
                         f"double-double evaluator, single thread, {el:.1f} s"}
        log(f"[bench] cpu oracle: {cpu['value']:.4e} evals/s ({reps} reps)")

    out = {
        "metric": "complex-dd monomial+gradient evals/s",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (complex double-double)",
        "data": "synthetic",
        "config": {"workload": "paper-scale system: n=128, 128 polynomials x m=256 monomials, "
                               "k=16, exponents 1..3, one point per step, graph-captured launches",
                   "n_vars": n, "n_polys": npoly, "monomials": M, "k": k,
                   "points_per_step": 1, "schedule": sched},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": traffic,
                     "traffic_unit": "bytes per evaluation (HBM, scaled FETCH_SIZE + WRITE_SIZE)",
                     "kernel": "eval_kernel<ArithDD>" + (" + combine_kernel<ArithDD>"
                                                         if sched["groups"] > 1 else ""),
                     "kernel_us": kern_ms * 1e3,
                     "flops_per_launch": flops, "flops_per_monomial": dd_flops_per_monomial(k),
                     "fp64_instr_rate_T": instr_rate,
                     "fp64_instr_frac": instr_rate / PEAK_FP64_TINSTR},
        "cpu_baseline": cpu,
        "side": side,
    }
    print(json.dumps(out), flush=True)


def copy_calibration(torch):
    """A plain copy of COPY_BYTES between two device buffers, 8 times, as an
    elementwise kernel (multiply by one: reads COPY_BYTES, writes COPY_BYTES;
    a same-dtype copy_ could go to a DMA engine instead of a kernel).  The
    counters of these dispatches against the known byte count give the scale
    of FETCH_SIZE and WRITE_SIZE."""
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(8):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "copies": 8,
                      "copy_kib": COPY_BYTES / 1024}), flush=True)


def measure_fp64(S, step, stream, M):
    import torch
    import paper_1201_0499_amd as pe
    for _ in range(50):
        step(pe.PE_FP64)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        for _ in range(GRAPH_LAUNCHES):
            step(pe.PE_FP64)
    g.replay()
    torch.cuda.synchronize()
    ms = timed(g.replay, 20) / GRAPH_LAUNCHES
    sched = S.get_schedule(1)
    log(f"[bench] fp64: {ms*1e3:.2f} us/step, {M/(ms*1e-3):.4e} evals/s, schedule {sched}")
    return {"fp64_evals_per_s": M / (ms * 1e-3), "fp64_us_per_step": ms * 1e3,
            "fp64_schedule": sched}


def measure_newton(pe, torch, stream, large=False):
    import synth
    if large:
        sys_np, xstar, starts = synth.newton_large_workload()
        desc = "known-root system n=512, m=1024+1, k=32, exponents 1..5"
    else:
        sys_np, xstar, starts = synth.newton_workload()
        desc = "known-root system n=128, m=256+1, k=16, exponents 1..3"
    n_starts = starts[0].shape[0]
    S = pe.System.from_csr(sys_np)
    out = {"workload": f"{desc}, {n_starts} starts at 1e-6, tol 1e-28", "starts": n_starts}
    for name, mode in (("mixed", pe.PE_NEWTON_MIXED), ("dd", pe.PE_NEWTON_DD)):
        best = None
        for rep in range(2):   # first run allocates the workspace
            x = tuple(torch.from_numpy(a).cuda() for a in starts)
            res = torch.zeros(n_starts, dtype=torch.float64, device="cuda")
            it = torch.zeros(n_starts, dtype=torch.int32, device="cuda")
            st = torch.zeros(n_starts, dtype=torch.int32, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S.newton(n_starts, x, res, it, st, tol=1e-28, max_iter=10, mode=mode, stream=stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            conv = int((st == 0).sum().item())
            if best is None or wall < best[0]:
                best = (wall, conv, float(res.max().item()), np.bincount(it.cpu().numpy()).tolist())
        wall, conv, rmax, hist = best
        out[name] = {"solves_per_s": conv / wall, "seconds": wall, "converged": conv,
                     "max_residual": rmax, "iterations_histogram": hist}
        log(f"[bench] newton{' large' if large else ''} {name}: {conv}/{n_starts} converged "
            f"in {wall*1e3:.1f} ms "
            f"-> {conv/wall:.1f} solves/s, max res {rmax:.2e}")
    out["mixed_over_dd"] = out["mixed"]["solves_per_s"] / max(out["dd"]["solves_per_s"], 1e-30)
    S.close()
    return out


def measure_batch(pe, torch, stream, cache):
    import synth
    systems, pts = synth.batch_workload()
    S = [pe.System.from_csr(s) for s in systems]
    B = pe.Batch(S)
    pps = np.array([p[0].shape[0] for p in pts], np.int64)
    xo, fo, jo = B.layout(pps)
    x = tuple(torch.from_numpy(np.concatenate([p[q].reshape(-1) for p in pts])).cuda() for q in range(4))
    f = tuple(torch.empty(int(fo[-1]), dtype=torch.float64, device="cuda") for _ in range(4))
    J = tuple(torch.empty(int(jo[-1]), dtype=torch.float64, device="cuda") for _ in range(4))
    evals = int(sum(s.n_monos * p[0].shape[0] for s, p in zip(systems, pts)))
    flops = int(sum(s.n_monos * p[0].shape[0] * dd_flops_per_monomial(s.max_k)
                    for s, p in zip(systems, pts)))
    t0 = time.perf_counter()
    B.autotune(pps, x, f, J, pe.PE_DD, stream=stream, cache_path=cache)
    tune_s = time.perf_counter() - t0
    B.eval_jac(pps, x, f, J, pe.PE_DD, stream=stream)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        B.eval_jac(pps, x, f, J, pe.PE_DD, stream=stream)
    g.replay()
    torch.cuda.synchronize()
    ms = timed(g.replay, 5)
    out = {"workload": "64 systems, n 16..256, m 16..1024, k 2..16, exponents 1..4, "
                       "64 points each; one graph-captured persistent launch",
           "evals": evals, "ms_per_launch": ms, "evals_per_s": evals / (ms * 1e-3),
           "tflops_algorithmic": flops / (ms * 1e-3) / 1e12,
           "frac_fp64_peak": flops / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
           "config": B.config(), "tune_seconds": tune_s}
    log(f"[bench] batch: {ms:.2f} ms/launch, {out['evals_per_s']:.4e} evals/s, "
        f"{out['tflops_algorithmic']:.2f} TFLOP/s, config {out['config']}")
    B.close()
    for s in S:
        s.close()
    return out


def measure_qd(pe, torch, stream, sys_np, pts):
    """Complex quad-double evaluation (pe_eval_jac_qd) of the headline system
    at its point (the dd point with zero lower words), HIP events over 200
    evaluations on the launch stream."""
    S = pe.System.from_csr(sys_np)
    n, npoly, M = sys_np.n_vars, sys_np.n_polys, sys_np.n_monos
    zero = np.zeros_like(pts[0])
    planes = [pts[0], pts[1], zero, zero, pts[2], pts[3], zero, zero]
    xq = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in planes]
    fq = [torch.empty((1, npoly), dtype=torch.float64, device="cuda") for _ in range(8)]
    Jq = [torch.empty((1, n, npoly), dtype=torch.float64, device="cuda") for _ in range(8)]
    for _ in range(10):
        S.eval_jac_qd(1, xq, fq, Jq, stream)
    torch.cuda.synchronize()
    reps = 200
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        S.eval_jac_qd(1, xq, fq, Jq, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    S.close()
    log(f"[bench] quad-double: {us:.2f} us/evaluation, {M / (us * 1e-6):.4e} evals/s")
    return {"workload": "headline system and point, complex quad-double", "us_per_evaluation": us,
            "evals_per_s": M / (us * 1e-6)}


def measure_paper_layout(pe, torch, stream, sys_np, x, f, J, fused_us):
    """The paper's three-kernel evaluation (pe_eval_jac_paper_layout) of the
    headline system at its point, timed like the headline (HIP events over
    repeated launches on the same stream), against the fused kernel."""
    S = pe.System.from_csr(sys_np)
    for _ in range(20):
        S.eval_jac_paper_layout(1, x, f, J, pe.PE_DD, stream)
    torch.cuda.synchronize()
    reps = 500
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        S.eval_jac_paper_layout(1, x, f, J, pe.PE_DD, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    S.close()
    dense = sys_np.n_monos * (sys_np.n_vars + 1) * 32
    log(f"[bench] paper layout (3 kernels, dense terms): {us:.2f} us/evaluation "
        f"({us / fused_us:.2f}x the fused kernel), dense array {dense / 2**20:.0f} MiB")
    return {"workload": "headline system and point, complex dd", "us_per_evaluation": us,
            "fused_us_per_evaluation": fused_us, "ratio": us / fused_us,
            "dense_array_bytes": dense}


def measure_track(pe, torch, stream):
    """Path tracking (pe_track): every total-degree path of the quadric
    tracking workload, with the double-double endgame."""
    import synth
    sys_np = synth.tracking_workload()
    n = sys_np.n_vars
    P = 2 ** n
    S = pe.System.from_csr(sys_np)
    best = None
    for rep in range(2):   # the first run allocates the workspace
        x = tuple(torch.empty((P, n), dtype=torch.float64, device="cuda") for _ in range(4))
        t = torch.zeros(P, dtype=torch.float64, device="cuda")
        res = torch.zeros(P, dtype=torch.float64, device="cuda")
        steps = torch.zeros(P, dtype=torch.int32, device="cuda")
        st = torch.zeros(P, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.start_solutions(0, P, x, stream=stream)
        S.track(P, x, t, steps, st, res, stream=stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if best is None or wall < best[0]:
            stc = st.cpu().numpy()
            best = (wall, int((stc == 0).sum()), float(steps.float().mean().item()),
                    int(steps.max().item()), float(res.max().item()))
    wall, ok, mean_steps, max_steps, rmax = best
    S.close()
    log(f"[bench] track: {ok}/{P} paths to roots in {wall*1e3:.1f} ms -> {ok/wall:.1f} paths/s, "
        f"mean {mean_steps:.1f} steps, max residual {rmax:.2e}")
    return {"workload": f"quadrics, n={n}: x_i^2 + 3 products + 2 linear terms + constant, "
                        f"all {P} total-degree paths, dd endgame to 1e-28",
            "paths": P, "reached": ok, "seconds": wall, "paths_per_s": ok / wall,
            "mean_steps": mean_steps, "max_steps": max_steps, "max_residual": rmax}


def measure_large(pe, torch, stream):
    import synth
    sys_np, pts = synth.large_workload()
    S = pe.System.from_csr(sys_np)
    P, n, npoly, M = pts[0].shape[0], sys_np.n_vars, sys_np.n_polys, sys_np.n_monos
    x = tuple(torch.from_numpy(a).cuda() for a in pts)
    f = tuple(torch.empty((P, npoly), dtype=torch.float64, device="cuda") for _ in range(4))
    J = tuple(torch.empty((P, n, npoly), dtype=torch.float64, device="cuda") for _ in range(4))
    out = {"workload": "n=512, 512 polynomials x m=1024 monomials, k=32, exponents 1..5, "
                       "256 points per launch", "schedule": S.get_schedule(P)}
    for name, prec in (("dd", pe.PE_DD), ("fp64", pe.PE_FP64)):
        S.eval_jac(P, x, f, J, prec, stream)
        torch.cuda.synchronize()
        ms = timed(lambda: S.eval_jac(P, x, f, J, prec, stream), 3)
        ev = M * P / (ms * 1e-3)
        out[name] = {"ms_per_launch": ms, "evals_per_s": ev}
        if prec == pe.PE_DD:
            tf = ev * dd_flops_per_monomial(32) / 1e12
            out[name]["tflops_algorithmic"] = tf
            out[name]["frac_fp64_peak"] = tf / PEAK_FP64_TFLOPS
        log(f"[bench] large {name}: {ms:.2f} ms/launch, {ev:.4e} evals/s")
    S.close()
    return out


if __name__ == "__main__":
    main()
