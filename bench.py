"""Throughput of the evaluation hot path on one MI355X.

Workload (the paper-scale configuration): a random system with n = 128
variables, 128 polynomials of m = 256 monomials, k = 16 variables per
monomial, exponents uniform in 1..3, unit-circle complex double-double
coefficients and point.  One step = one evaluation of the system and its
full Jacobian in complex double-double at one point (one pe_eval_jac call),
repeated as in Newton iterations.  Inputs are resident in HBM before the
timed region; nothing is skipped inside it.

Prints one JSON line: complex-dd monomial+gradient evaluations per second,
the roofline of the evaluation kernel (FP64 vector ALU bound), the oracle's
CPU throughput on a bounded sample, and side measurements.
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

PEAK_FP64_TFLOPS = 78.6          # MI355X FP64 vector, FMA = 2 flops
# algorithmic FP64 flops per monomial for value + all k partials in complex dd:
# (6k-5) complex dd products (88 flops) + (k+1) complex dd sums (40 flops)
def dd_flops_per_monomial(k: int) -> int:
    return 568 * k - 400


def fp64_flops_per_monomial(k: int) -> int:
    # (6k-5) complex products (6 flops) + (k+1) complex sums (2 flops)
    return 38 * k - 28


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--skip-side", action="store_true", help="only the headline measurement")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import synth
    import paper_1201_0499_amd as pe

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    sys_np, pts = synth.paper_scale_workload()
    n, npoly, M, k = sys_np.n_vars, sys_np.n_polys, sys_np.n_monos, sys_np.max_k
    log(f"[bench] workload n={n} polys={npoly} monomials={M} k={k} max_exp={sys_np.max_exp}")
    S = pe.System.from_csr(sys_np)
    x = tuple(torch.from_numpy(a).to(dev) for a in pts)
    f = tuple(torch.empty((1, npoly), dtype=torch.float64, device=dev) for _ in range(4))
    J = tuple(torch.empty((1, n, npoly), dtype=torch.float64, device=dev) for _ in range(4))
    stream = torch.cuda.current_stream()
    sched = S.get_schedule(1)
    log(f"[bench] schedule {sched}")

    def step(prec=pe.PE_DD):
        S.eval_jac(1, x, f, J, prec, stream)

    # ---- warmup ----
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # ---- timed region: exactly K steps ----
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    ms_per_step = 1e3 * wall / args.steps
    value = M * args.steps / wall
    log(f"[bench] dd: {ms_per_step*1e3:.2f} us/step, {value:.4e} evals/s")

    # ---- kernel duration with HIP events on the launch stream ----
    n_ev = min(args.steps, 2000)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(n_ev)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(n_ev)]
    for i in range(n_ev):
        starts[i].record(stream)
        step()
        ends[i].record(stream)
    torch.cuda.synchronize()
    kern_ms = float(np.mean([s.elapsed_time(e) for s, e in zip(starts, ends)]))
    flops = M * dd_flops_per_monomial(k)
    achieved = flops / (kern_ms * 1e-3) / 1e12
    log(f"[bench] dd kernel {kern_ms*1e3:.2f} us/launch (events), {achieved:.2f} TFLOP/s algorithmic")

    side = {}
    if not args.skip_side:
        # FP64 mode on the same workload
        for _ in range(100):
            step(pe.PE_FP64)
        torch.cuda.synchronize()
        K64 = max(100, args.steps // 2)
        t0 = time.perf_counter()
        for _ in range(K64):
            step(pe.PE_FP64)
        torch.cuda.synchronize()
        w64 = time.perf_counter() - t0
        side["fp64_evals_per_s"] = M * K64 / w64
        side["fp64_us_per_step"] = 1e6 * w64 / K64
        log(f"[bench] fp64: {1e6*w64/K64:.2f} us/step, {M*K64/w64:.4e} evals/s")

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
        cpu = {"value": M * reps / el, "unit": "complex-dd monomial+gradient evals/s",
               "cores": 1, "kind": "oracle",
               "sample": f"{reps} full evaluations of the same system and point "
                         f"({reps * M} monomials with all partials), definitional dd "
                         f"evaluator, single thread, {el:.1f} s"}
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
                               "k=16, exponents 1..3, one point per step",
                   "n_vars": n, "n_polys": npoly, "monomials": M, "k": k,
                   "points_per_step": 1, "schedule": sched},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                     "kernel_us": kern_ms * 1e3,
                     "flops_per_launch": flops,
                     "flops_per_monomial": dd_flops_per_monomial(k)},
        "cpu_baseline": cpu,
        "side": side,
    }
    S.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
