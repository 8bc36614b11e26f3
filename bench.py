"""Throughput of the evaluation hot path on one MI355X.

Headline workload (the largest single-GPU configuration): a system of
n = 512 variables and 512 polynomials of m = 1024 monomials, k = 32
variables per monomial, exponents uniform in 1..5, unit-circle complex
double-double coefficients, evaluated with its full Jacobian at 256
unit-circle points per launch.  One step = one pe_eval_jac call over the 256
points (one kernel launch), with the schedule chosen by the library's
autotuner (pe_autotune_system, cached in a text file).  Inputs are resident
in HBM before the timed region; the timed region is exactly --steps launches
between two device synchronizations, and HIP events recorded on the launch
stream around it give the GPU time per launch.

Side measurements (same JSON line, "side"):
  * the paper-scale system (n=128, m=256, k=16, exponents 1..3) at one point
    per launch, 10,000 launches replayed from a hipGraph, double-double and
    FP64, with its own roofline;
  * the headline system in FP64;
  * Newton on known-root systems (n=128, m=256+1, k=16, 1024 starts, and
    n=512, m=1024+1, k=32, 256 starts) to max|f| < 1e-28: solves/s in mixed
    precision and in all double-double; at n=128 also the quad-double
    corrector (pe_newton_qd) to max|f| < 1e-56;
  * a batch of 64 uneven systems in one autotuned, graph-captured persistent
    launch; path tracking; the paper's three-kernel organisation; quad-double.

The CPU baseline is the oracle's fast mode (power table, common factor,
prefix/suffix products; OpenMP over (point, polynomial) pairs) on every host
thread OpenMP is given, on a bounded sample of the headline workload, with
its one-thread rate and the definitional evaluator's beside it.

Prints one JSON line on stdout; progress goes to stderr.

``--counters DIR`` (no GPU) turns the CSV output of rocprofv3 counter runs
of the headline command into the record this script reads its executed
FP64 instruction count and HBM traffic from.
"""
from __future__ import annotations

import argparse
import glob
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector (FMA counted as 2 flops)
PEAK_FP64_TINSTR = 39.3      # FP64 lane-instructions/s: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz
PEAK_HBM_GBS = 8000.0
GRAPH_LAUNCHES = 100
C2_LAUNCHES = 10000          # the paper-scale workload is repeated 10,000 times
COPY_BYTES = 512 << 20       # copy-calibration size

HEADLINE_RECORD = os.path.join(ROOT, "profiles", "eval_kernel_dd_large_counters.json")
TUNED_SCHEDULES = os.path.join(ROOT, "paper_1201_0499_amd", "tuned_schedules.txt")
C2_RECORD = os.path.join(ROOT, "profiles", "eval_kernel_dd_paper_scale_traffic.json")

# The paper's own measurements (Section 4, Tables 1 and 2): systems of
# dimension 32 evaluated 100,000 times with their Jacobians, one point at a
# time, on an NVIDIA Tesla C2050 against one core of an Intel Xeon X5690; the
# tables do not state the precision (the kernels are described in complex
# double).  evals/s = monomials x 1e5 / seconds.
PAPER_C2050 = {
    "source": "Section 4, Tables 1 and 2",
    "gpu": "NVIDIA Tesla C2050, 14 multiprocessors x 32 cores at 1147 MHz, CUDA 4.0",
    "cpu": "one core of an Intel Xeon X5690 at 3.47 GHz",
    "workload": "n = 32, 100,000 evaluations of f and J, one point per evaluation",
    "precision": "not stated; the kernels are described in complex double",
    "rows": [
        {"monomials": m, "k": k, "max_exp": d, "gpu_s": g, "cpu_s": c,
         "gpu_evals_per_s": m * 1e5 / g, "cpu_evals_per_s": m * 1e5 / c}
        for (m, k, d, g, c) in [(704, 9, 2, 14.514, 110.9), (1024, 9, 2, 15.265, 159.3),
                                (1536, 9, 2, 17.000, 238.7), (704, 16, 10, 19.068, 196.9),
                                (1024, 16, 10, 20.800, 283.3), (1536, 16, 10, 21.763, 425.8)]
    ],
}


def dd_flops_per_monomial(k: int) -> int:
    """Algorithmic flops of value + all k partials of one monomial in complex
    double-double, the paper's method: (6k-5) complex dd products of 88
    flops (four double-word products, two double-word sums) and (k+1)
    complex dd sums of 40 flops."""
    return 568 * k - 400


def f64_flops_per_monomial(k: int) -> int:
    """The same in complex FP64: (6k-5) complex products of 6 flops and
    (k+1) complex sums of 2."""
    return 38 * k - 28


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_name(arith, sched):
    """Name of the evaluation kernel instantiation a schedule launches (its
    workgroup-size bound is 256, 512 or 1024)."""
    nt = sched["threads"]
    maxt = 256 if nt <= 256 else (512 if nt <= 512 else 1024)
    return f"eval_kernel<{arith}, {sched['chunk_vars']}, {maxt}>"


def kernel_sources_sha256():
    """Hash of the sources that decide the evaluation kernel and its launch:
    eval.hip, the schedule tables (schedule.cpp), the launch code (api.cpp)
    and the headers of those three that define the evaluation.  A change to
    the Newton, tracker, batch or ablation code leaves the evaluation's
    counters valid."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1201_0499_amd", "csrc")
    for f in ("api.cpp", "dd.hpp", "device.hpp", "eval.hip", "eval.hpp", "internal.hpp",
              "monomial.hpp", "packing.hpp", "qd.hpp", "schedule.cpp", "schedule.hpp"):
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_record(path, sched, kernel_prefix):
    """The committed counter record's entry for the kernel whose name starts
    with kernel_prefix, or None when the record is missing or was taken
    with other kernel sources or another schedule."""
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("sources_sha256") != kernel_sources_sha256() or rec.get("schedule") != sched:
        return None
    for name, v in rec.get("kernels", {}).items():
        if name.startswith(kernel_prefix):
            return dict(v, fetch_scale=rec.get("fetch_scale"), write_scale=rec.get("write_scale"))
    return None


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


def roofline_block(kernel, sched, seconds, flops, rec):
    """The roofline object of one kernel: algorithmic flops per launch over the
    measured time per launch, against FP64 vector peak; the executed FP64
    mix and the HBM traffic from the counter record when it matches."""
    achieved = flops / seconds / 1e12
    out = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
           "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
           "traffic_unit": "bytes per launch (HBM: FETCH_SIZE and WRITE_SIZE, each scaled by "
                           "what it reads for a copy of known size)",
           "kernel": kernel, "schedule": sched, "kernel_us": seconds * 1e6,
           "flops_per_launch": flops,
           "achieved_kind": "algorithmic: the paper's operation count per monomial "
                            "(see flops_per_monomial) x monomials x points / time per launch"}
    if rec is not None:
        fs, ws = rec["fetch_scale"], rec["write_scale"]
        out["traffic"] = rec["fetch_kib"] * 1024 * fs + rec["write_kib"] * 1024 * ws
        out["hbm_gbs"] = out["traffic"] / seconds / 1e9
        out["hbm_frac"] = out["hbm_gbs"] / PEAK_HBM_GBS
        lanes = 64.0
        instr = (rec["add_f64"] + rec["mul_f64"] + rec["fma_f64"]) * lanes
        eflops = (rec["add_f64"] + rec["mul_f64"] + 2.0 * rec["fma_f64"]) * lanes
        out["executed"] = {
            "source": "rocprofv3 SQ_INSTS_VALU_{ADD,MUL,FMA}_F64 per dispatch x 64 lanes",
            "fp64_lane_instr_per_launch": instr,
            "fp64_instr_rate_T": instr / seconds / 1e12,
            "fp64_instr_frac": instr / seconds / 1e12 / PEAK_FP64_TINSTR,
            "tflops": eflops / seconds / 1e12,
            "frac": eflops / seconds / 1e12 / PEAK_FP64_TFLOPS}
    return out


# ---------------------------------------------------------------------------
# headline: the large system at 256 points, complex double-double
# ---------------------------------------------------------------------------

def measure_headline(pe, torch, stream, args):
    import synth
    sys_np, pts = synth.large_workload()
    P, n, npoly, M, k = pts[0].shape[0], sys_np.n_vars, sys_np.n_polys, sys_np.n_monos, sys_np.max_k
    log(f"[bench] headline workload n={n} polys={npoly} monomials={M} k={k} "
        f"max_exp={sys_np.max_exp} points={P}")
    S = pe.System.from_csr(sys_np)
    dev = torch.device("cuda:0")
    x = tuple(torch.from_numpy(a).to(dev) for a in pts)
    f = tuple(torch.empty((P, npoly), dtype=torch.float64, device=dev) for _ in range(4))
    J = tuple(torch.empty((P, n, npoly), dtype=torch.float64, device=dev) for _ in range(4))
    t0 = time.perf_counter()
    if not args.no_tune:
        S.autotune(P, x, f, J, pe.PE_DD, stream=stream, cache_path=args.tune_cache)
    sched = S.get_schedule(P)
    log(f"[bench] schedule {sched} (tuning {time.perf_counter() - t0:.1f} s)")

    def step(prec=pe.PE_DD):
        S.eval_jac(P, x, f, J, prec, stream)

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    # ---- timed region: exactly --steps launches ----
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_s = ev0.elapsed_time(ev1) * 1e-3 / args.steps
    value = M * P * args.steps / wall
    log(f"[bench] dd: {wall / args.steps * 1e3:.3f} ms/step (wall), {gpu_s * 1e3:.3f} ms "
        f"(events), {value:.4e} evals/s")
    flops = M * P * dd_flops_per_monomial(k)
    rec = counter_record(HEADLINE_RECORD, sched, "void pe::eval_kernel<pe::ArithDD")
    roof = roofline_block(kernel_name("ArithDD", sched), sched, gpu_s, flops, rec)
    roof["flops_per_monomial"] = dd_flops_per_monomial(k)
    log(f"[bench] dd roofline: {roof['achieved']:.2f} TFLOP/s algorithmic = "
        f"{roof['frac']:.3f} of FP64 peak"
        + (f"; executed {roof['executed']['fp64_instr_frac']:.3f} of FP64 issue, "
           f"HBM {roof['hbm_gbs']:.0f} GB/s" if rec else "; no matching counter record"))

    side = {}
    if not args.skip_side:
        # the same system and points in FP64 (its own tuned schedule)
        if not args.no_tune:
            S.autotune(P, x, f, J, pe.PE_FP64, stream=stream, cache_path=args.tune_cache)
        step(pe.PE_FP64)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record(stream)
        for _ in range(reps):
            step(pe.PE_FP64)
        e1.record(stream)
        torch.cuda.synchronize()
        s64 = e0.elapsed_time(e1) * 1e-3 / reps
        sch64 = S.get_schedule(P)
        side["large_fp64"] = {
            "workload": "headline system and points, complex FP64", "ms_per_launch": s64 * 1e3,
            "evals_per_s": M * P / s64,
            "roofline": roofline_block(kernel_name("Arith64", sch64), sch64, s64,
                                       M * P * f64_flops_per_monomial(k), None)}
        side["large_fp64"]["roofline"]["flops_per_monomial"] = f64_flops_per_monomial(k)
        log(f"[bench] large fp64: {s64 * 1e3:.3f} ms/launch, {M * P / s64:.4e} evals/s, "
            f"{side['large_fp64']['roofline']['frac']:.3f} of FP64 peak, schedule {sch64}")
    S.close()
    head = {"value": value, "ms_per_step": 1e3 * wall / args.steps, "roofline": roof,
            "config": {"workload": "large system: n=512, 512 polynomials x m=1024 monomials, "
                                   "k=32, exponents 1..5, 256 points per step (one launch), "
                                   "complex double-double, f and full Jacobian",
                       "n_vars": n, "n_polys": npoly, "monomials": M, "k": k,
                       "points_per_step": P, "schedule": sched}}
    return head, side, sys_np, pts


# ---------------------------------------------------------------------------
# CPU baseline: the oracle's fast mode on the host
# ---------------------------------------------------------------------------

def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def measure_cpu(sys_np, pts, seconds):
    from oracle import ddoracle as O
    M = sys_np.n_monos
    P = pts[0].shape[0]
    # all threads OpenMP is given: whole points, until the time is spent
    t0 = time.perf_counter()
    done, used = 0, 1
    while True:
        one = tuple(a[done:done + 1] for a in pts)
        _, _, used = O.eval_dd_fast(sys_np, one)
        done += 1
        el = time.perf_counter() - t0
        if el >= seconds or done >= P:
            break
    rate_all = M * done / el
    log(f"[bench] cpu oracle fast mode, {used} threads: {rate_all:.4e} evals/s "
        f"({done} points in {el:.1f} s)")
    # one thread: the first polynomials of the first point, about seconds/4
    one = tuple(a[:1] for a in pts)
    t0 = time.perf_counter()
    O.eval_dd_fast(sys_np, one, polys=list(range(4)), threads=1)
    probe = time.perf_counter() - t0
    nsel = int(min(sys_np.n_polys, max(4, 4 * (seconds / 4) / max(probe, 1e-6))))
    t0 = time.perf_counter()
    O.eval_dd_fast(sys_np, one, polys=list(range(nsel)), threads=1)
    el1 = time.perf_counter() - t0
    mono_sel = int(sys_np.poly_start[nsel])
    rate_1 = mono_sel / el1
    log(f"[bench] cpu oracle fast mode, 1 thread: {rate_1:.4e} evals/s ({nsel} polynomials)")
    # the definitional evaluator, one thread, two polynomials
    t0 = time.perf_counter()
    O.eval_dd(sys_np, one, polys=[0, 1])
    eln = time.perf_counter() - t0
    rate_n = int(sys_np.poly_start[2]) / eln
    log(f"[bench] cpu oracle definitional, 1 thread: {rate_n:.4e} evals/s")
    return {"value": rate_all, "unit": "evals/s", "cores": used, "kind": "oracle",
            "mode": "fast (power table, common factor, prefix/suffix products), OpenMP over "
                    "(point, polynomial) pairs",
            "sample": f"{done} of the {P} points of the headline workload, all outputs, "
                      f"{el:.1f} s on {used} threads",
            "host": {"cpu_model": cpu_model(), "nproc": os.cpu_count(),
                     "omp_num_threads": os.environ.get("OMP_NUM_THREADS")},
            "single_core": {"value": rate_1, "unit": "evals/s",
                            "sample": f"first {nsel} polynomials at one point, {el1:.1f} s"},
            "definitional_single_core": {"value": rate_n, "unit": "evals/s",
                                         "sample": f"2 polynomials at one point, {eln:.1f} s"}}


# ---------------------------------------------------------------------------
# side measurements
# ---------------------------------------------------------------------------

def measure_paper_scale(pe, torch, stream, args):
    """The paper-scale system at one point per launch: 10,000 launches
    replayed from a hipGraph of 100, HIP events around the replays."""
    import synth
    sys_np, pts = synth.paper_scale_workload()
    n, npoly, M, k = sys_np.n_vars, sys_np.n_polys, sys_np.n_monos, sys_np.max_k
    S = pe.System.from_csr(sys_np)
    x = tuple(torch.from_numpy(a).cuda() for a in pts)
    f = tuple(torch.empty((1, npoly), dtype=torch.float64, device="cuda") for _ in range(4))
    J = tuple(torch.empty((1, n, npoly), dtype=torch.float64, device="cuda") for _ in range(4))
    out = {"workload": "paper-scale system: n=128, 128 polynomials x m=256 monomials, k=16, "
                       "exponents 1..3, one point per launch, 10,000 launches from a hipGraph"}
    for name, prec in (("dd", pe.PE_DD), ("fp64", pe.PE_FP64)):
        if not args.no_tune:
            S.autotune(1, x, f, J, prec, stream=stream, cache_path=args.tune_cache)
        sched = S.get_schedule(1)
        for _ in range(50):
            S.eval_jac(1, x, f, J, prec, stream)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            for _ in range(GRAPH_LAUNCHES):
                S.eval_jac(1, x, f, J, prec, stream)
        with torch.cuda.stream(stream):
            g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            t0 = time.perf_counter()
            e0.record(stream)
            for _ in range(C2_LAUNCHES // GRAPH_LAUNCHES):
                g.replay()
            e1.record(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        s = e0.elapsed_time(e1) * 1e-3 / C2_LAUNCHES
        per = dd_flops_per_monomial(k) if prec == pe.PE_DD else f64_flops_per_monomial(k)
        kname = ("eval_kernel<ArithDD>" if prec == pe.PE_DD else "eval_kernel<Arith64>") + \
            (" + combine_kernel" if sched["groups"] > 1 else "")
        rec = None
        if prec == pe.PE_DD:
            rec = c2_traffic_record(sched)
        roof = roofline_block(kname, sched, s, M * per, rec)
        roof["flops_per_monomial"] = per
        out[name] = {"us_per_evaluation": s * 1e6, "us_per_evaluation_wall": wall / C2_LAUNCHES * 1e6,
                     "evals_per_s": M / s, "roofline": roof}
        log(f"[bench] paper-scale {name}: {s * 1e6:.2f} us/evaluation (events), "
            f"{M / s:.4e} evals/s, {roof['frac']:.3f} of FP64 peak, schedule {sched}")
        if prec == pe.PE_DD:
            out[name]["new_point_per_launch"] = paper_scale_moving_point(pe, torch, stream, S, M, f, J)
            out[name]["end_to_end"] = paper_scale_end_to_end(pe, torch, stream, S, M, pts, f, J)
    S.close()
    return out, sys_np, pts, x, f, J


def paper_scale_moving_point(pe, torch, stream, S, M, f, J, n_pts=100):
    """The same dd evaluation with a different point at every launch: a
    hipGraph of 100 launches over 100 seeded unit-circle points, replayed
    100 times (10,000 launches), HIP events around the replays."""
    import synth
    n = S.n_vars
    xs = tuple(torch.from_numpy(a).cuda() for a in synth.points(n_pts, n, synth.config_seed(1, 1)))
    views = [tuple(t[j:j + 1] for t in xs) for j in range(n_pts)]
    for v in views:
        S.eval_jac(1, v, f, J, pe.PE_DD, stream)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        for v in views:
            S.eval_jac(1, v, f, J, pe.PE_DD, stream)
    reps = C2_LAUNCHES // n_pts
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        g.replay()
        e0.record(stream)
        for _ in range(reps):
            g.replay()
        e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / (reps * n_pts)
    log(f"[bench] paper-scale dd, a new point per launch: {us:.2f} us/evaluation (events)")
    return {"points": n_pts, "us_per_evaluation": us, "evals_per_s": M / (us * 1e-6)}


def paper_scale_end_to_end(pe, torch, stream, S, M, pts, f, J, reps=1000):
    """The dd evaluation with its transfers, as a host program would run it:
    per evaluation the point goes from pinned host memory to the device and
    f and J come back to pinned host memory, all on the launch stream; wall
    time over 1000 evaluations between two synchronizations."""
    hx = tuple(torch.from_numpy(a).pin_memory() for a in pts)
    dx = tuple(torch.empty_like(t, device="cuda") for t in hx)
    hf = tuple(torch.empty(t.shape, dtype=t.dtype).pin_memory() for t in f)
    hJ = tuple(torch.empty(t.shape, dtype=t.dtype).pin_memory() for t in J)

    def one():
        with torch.cuda.stream(stream):
            for d, h in zip(dx, hx):
                d.copy_(h, non_blocking=True)
            S.eval_jac(1, dx, f, J, pe.PE_DD, stream)
            for h, d in zip(hf + hJ, f + J):
                h.copy_(d, non_blocking=True)

    for _ in range(20):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        one()
    torch.cuda.synchronize()
    us = (time.perf_counter() - t0) * 1e6 / reps
    moved = sum(t.numel() * 8 for t in hx + hf + hJ)
    log(f"[bench] paper-scale dd with transfers: {us:.2f} us/evaluation (wall), "
        f"{moved / 1024:.0f} KiB moved per evaluation")
    return {"us_per_evaluation_wall": us, "evals_per_s": M / (us * 1e-6),
            "bytes_moved_per_evaluation": moved,
            "what": "H2D of the point and D2H of f and J through pinned host buffers, on the "
                    "launch stream, per evaluation; not graph-captured"}


def c2_traffic_record(sched):
    """HBM bytes of the paper-scale dd evaluation from its committed record,
    in the form counter_record returns (summed over its kernels)."""
    try:
        with open(C2_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("sources_sha256") != kernel_sources_sha256() or rec.get("schedule") != sched:
        return None
    ks = rec.get("kernels", {}).values()
    tot = {key: sum(v.get(key, 0.0) for v in ks) for key in ("fetch_kib", "write_kib", "add_f64",
                                                              "mul_f64", "fma_f64")}
    if not all(("add_f64" in v) for v in ks):
        return None
    return dict(tot, fetch_scale=rec["fetch_scale"], write_scale=rec["write_scale"])


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
            f"in {wall*1e3:.1f} ms -> {conv/wall:.1f} solves/s, max res {rmax:.2e}")
    out["mixed_over_dd"] = out["mixed"]["solves_per_s"] / max(out["dd"]["solves_per_s"], 1e-30)
    if not large:
        out["qd"] = measure_newton_qd(torch, stream, S, starts)
    S.close()
    return out


def measure_newton_qd(torch, stream, S, starts, tol=1e-56):
    """pe_newton_qd (FP64 Jacobian and elimination, quad-double residual and
    iterate) from the same starts, to max_p |f_p| < 1e-56."""
    n_starts = starts[0].shape[0]
    z = np.zeros_like(starts[0])
    planes = [starts[0], starts[1], z, z, starts[2], starts[3], z, z]
    best = None
    for rep in range(2):   # first run allocates the workspace
        x = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in planes]
        res = torch.zeros(n_starts, dtype=torch.float64, device="cuda")
        it = torch.zeros(n_starts, dtype=torch.int32, device="cuda")
        st = torch.zeros(n_starts, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.newton_qd(n_starts, x, res, it, st, tol=tol, max_iter=12, stream=stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        conv = int((st == 0).sum().item())
        if best is None or wall < best[0]:
            best = (wall, conv, float(res.max().item()), np.bincount(it.cpu().numpy()).tolist())
    wall, conv, rmax, hist = best
    log(f"[bench] newton qd: {conv}/{n_starts} converged to {tol:.0e} in {wall*1e3:.1f} ms -> "
        f"{conv/wall:.1f} solves/s, max res {rmax:.2e}")
    return {"tol": tol, "solves_per_s": conv / wall, "seconds": wall, "converged": conv,
            "max_residual": rmax, "iterations_histogram": hist}


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
    out["k_buckets"] = batch_k_buckets(pe, torch, stream, systems, pts, S)
    for s in S:
        s.close()
    return out


def batch_k_buckets(pe, torch, stream, systems, pts, S, edges=((2, 5), (6, 10), (11, 16))):
    """The batch's systems grouped by k, one launch per group with the
    automatic batch configuration (no tuning), wall clock over 5 launches
    between two synchronizations."""
    rows = []
    for lo, hi in edges:
        idx = [i for i, s in enumerate(systems) if lo <= s.max_k <= hi]
        if not idx:
            continue
        B = pe.Batch([S[i] for i in idx])
        pps = np.array([pts[i][0].shape[0] for i in idx], np.int64)
        xo, fo, jo = B.layout(pps)
        x = tuple(torch.from_numpy(np.concatenate([pts[i][q].reshape(-1) for i in idx])).cuda()
                  for q in range(4))
        f = tuple(torch.empty(int(fo[-1]), dtype=torch.float64, device="cuda") for _ in range(4))
        J = tuple(torch.empty(int(jo[-1]), dtype=torch.float64, device="cuda") for _ in range(4))
        B.eval_jac(pps, x, f, J, pe.PE_DD, stream=stream)
        torch.cuda.synchronize()
        ms = timed(lambda: B.eval_jac(pps, x, f, J, pe.PE_DD, stream=stream), 5)
        evals = int(sum(systems[i].n_monos * pts[i][0].shape[0] for i in idx))
        flops = int(sum(systems[i].n_monos * pts[i][0].shape[0] *
                        dd_flops_per_monomial(systems[i].max_k) for i in idx))
        rows.append({"k": [lo, hi], "systems": len(idx), "evals": evals, "ms_per_launch": ms,
                     "evals_per_s": evals / (ms * 1e-3),
                     "frac_fp64_peak": flops / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS})
        log(f"[bench] batch k {lo}..{hi}: {len(idx)} systems, {ms:.2f} ms/launch, "
            f"{rows[-1]['evals_per_s']:.4e} evals/s, {rows[-1]['frac_fp64_peak']:.3f} of FP64 peak")
        B.close()
    return rows


def measure_qd(pe, torch, stream, sys_np=None, pts=None):
    """Complex quad-double evaluation (pe_eval_jac_qd) of the paper-scale
    system at its point (the dd point with zero lower words): HIP events over
    200 evaluations replayed from a hipGraph of 100 (the outputs of a replay
    checked bit for bit against an eager call), and over 200 evaluations
    launched from the host one by one."""
    if sys_np is None:
        import synth
        sys_np, pts = synth.paper_scale_workload()
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
    eager = [t.clone() for t in fq + Jq]
    reps = 200
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        for _ in range(reps // 2):
            S.eval_jac_qd(1, xq, fq, Jq, stream)
    for t in fq + Jq:
        t.fill_(float("nan"))
    with torch.cuda.stream(stream):
        g.replay()
    torch.cuda.synchronize()
    same = all(torch.equal(a.view(torch.int64), b.view(torch.int64)) for a, b in zip(fq + Jq, eager))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        e0.record(stream)
        g.replay()
        g.replay()
        e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    e0.record(stream)
    for _ in range(reps):
        S.eval_jac_qd(1, xq, fq, Jq, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    us_host = e0.elapsed_time(e1) * 1e3 / reps
    S.close()
    log(f"[bench] quad-double: {us:.2f} us/evaluation (graph replays; replay equals eager: {same}), "
        f"{M / (us * 1e-6):.4e} evals/s; {us_host:.2f} us launched one by one from the host")
    return {"workload": "paper-scale system and point, complex quad-double, 200 evaluations "
                        "replayed from a hipGraph of 100",
            "us_per_evaluation": us, "evals_per_s": M / (us * 1e-6),
            "replay_equals_eager": same, "us_per_evaluation_host_launched": us_host}


def measure_paper_layout(pe, torch, stream, sys_np, x, f, J, fused_us):
    """The paper's three-kernel evaluation (pe_eval_jac_paper_layout) of the
    paper-scale system at its point, HIP events over 500 launches on the
    stream, against the fused kernel."""
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
    return {"workload": "paper-scale system and point, complex dd", "us_per_evaluation": us,
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


def measure_fp64_eval(pe, torch, stream):
    """FP64 evaluation alone (for counter runs): the paper-scale known-root
    system at 1024 points (the mixed Newton's Jacobian at C3 size) and the
    large system at 256 points, 5 launches each."""
    import synth
    out = {}
    for name, (sys_np, P) in (("paper_scale_1024", (synth.newton_workload(n_starts=1)[0], 1024)),
                              ("large_256", (synth.large_workload(n_points=1)[0], 256))):
        n, npoly, M, k = sys_np.n_vars, sys_np.n_polys, sys_np.n_monos, sys_np.max_k
        pts = synth.points(P, n, 4242)
        S = pe.System.from_csr(sys_np)
        x = tuple(torch.from_numpy(a).cuda() for a in pts)
        f = tuple(torch.empty((P, npoly), dtype=torch.float64, device="cuda") for _ in range(4))
        J = tuple(torch.empty((P, n, npoly), dtype=torch.float64, device="cuda") for _ in range(4))
        S.eval_jac(P, x, f, J, pe.PE_FP64, stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            S.eval_jac(P, x, f, J, pe.PE_FP64, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        s = e0.elapsed_time(e1) * 1e-3 / 5
        mono = int(np.sum(np.diff(sys_np.mono_start) > 0))
        fl = mono * P * f64_flops_per_monomial(k)
        out[name] = {"ms_per_launch": s * 1e3, "schedule": S.get_schedule(P),
                     "tflops_algorithmic": fl / s / 1e12, "frac": fl / s / 1e12 / PEAK_FP64_TFLOPS}
        log(f"[bench] fp64 {name}: {s * 1e3:.3f} ms/launch, {out[name]['frac']:.3f} of FP64 peak")
        S.close()
    return out


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


# ---------------------------------------------------------------------------
# counter record from rocprofv3 CSV output (runs on the CPU)
# ---------------------------------------------------------------------------

def summarize_counters(root, out_json, workload, sched):
    """Read every *counter_collection.csv under root: one directory per
    counter run, named ``calib_*`` for runs of --copy-calibration.  Writes the
    per-kernel means per dispatch (KiB for FETCH_SIZE / WRITE_SIZE) and the
    copy scales to out_json, and prints a markdown table."""
    import csv
    vals = {}      # (kind, kernel, counter) -> list of per-dispatch values
    for path in glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True):
        kind = "calib" if "/calib" in path else "run"
        per = {}
        with open(path) as fh:
            for row in csv.DictReader(fh):
                key = (row["Kernel_Name"], row["Counter_Name"], row["Dispatch_Id"])
                per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
        for (kern, ctr, _), v in per.items():
            vals.setdefault((kind, kern, ctr), []).append(v)
    mean = {k: float(np.mean(v)) for k, v in vals.items()}
    copy_kib = COPY_BYTES / 1024
    calib = [k for k in mean if k[0] == "calib"]
    fetch_c = max((mean[k] for k in calib if k[2] == "FETCH_SIZE"), default=None)
    write_c = max((mean[k] for k in calib if k[2] == "WRITE_SIZE"), default=None)
    rec = {"workload": workload, "schedule": sched, "sources_sha256": kernel_sources_sha256(),
           "fetch_scale": copy_kib / fetch_c if fetch_c else None,
           "write_scale": copy_kib / write_c if write_c else None, "kernels": {}}
    names = {"FETCH_SIZE": "fetch_kib", "WRITE_SIZE": "write_kib",
             "SQ_INSTS_VALU_ADD_F64": "add_f64", "SQ_INSTS_VALU_MUL_F64": "mul_f64",
             "SQ_INSTS_VALU_FMA_F64": "fma_f64", "SQ_INSTS_VALU": "valu",
             "SQ_ACTIVE_INST_VALU": "active_inst_valu", "SQ_BUSY_CYCLES": "busy_cycles",
             "SQ_WAVES": "waves", "GRBM_GUI_ACTIVE": "gui_active",
             "SQ_LDS_BANK_CONFLICT": "lds_bank_conflict", "SQ_LDS_IDX_ACTIVE": "lds_idx_active",
             "SQ_INSTS_LDS": "insts_lds", "SQ_WAIT_INST_LDS": "wait_inst_lds",
             "SQ_WAIT_INST_ANY": "wait_inst_any", "SQ_WAVE_CYCLES": "wave_cycles"}
    for (kind, kern, ctr), v in mean.items():
        if kind != "run" or ctr not in names:
            continue
        rec["kernels"].setdefault(kern, {})[names[ctr]] = v
    with open(out_json, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(f"copy calibration: FETCH_SIZE scale {rec['fetch_scale']}, WRITE_SIZE scale "
          f"{rec['write_scale']}")
    cols = sorted({c for v in rec["kernels"].values() for c in v})
    print("| kernel | " + " | ".join(cols) + " |")
    print("|---|" + "---:|" * len(cols))
    for kern, v in sorted(rec["kernels"].items()):
        print(f"| `{kern}` | " + " | ".join(f"{v.get(c, float('nan')):.6g}" for c in cols) + " |")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--skip-side", action="store_true", help="only the headline measurement")
    ap.add_argument("--no-tune", action="store_true", help="automatic schedules, no search")
    ap.add_argument("--tune-cache", default=TUNED_SCHEDULES,
                    help="schedule cache read (and appended to) by the autotuners; the default "
                         "is the committed file of schedules tuned on an MI355X, which the GPU "
                         "parity tests of the measured configurations read too")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 512 MiB (8 times), the reference for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--only", choices=["paper_scale", "newton", "newton_large", "track",
                                       "fp64_eval", "batch", "quad_double"],
                    help="run one side measurement alone and print its JSON (for profiling)")
    ap.add_argument("--counters", metavar="DIR",
                    help="(no GPU) summarize rocprofv3 counter CSVs under DIR into --record")
    ap.add_argument("--record", default=HEADLINE_RECORD)
    ap.add_argument("--record-workload", default="large system (n=512, 512 polynomials x m=1024 "
                                                  "monomials, k=32, exponents 1..5), 256 points")
    ap.add_argument("--record-schedule", default=None,
                    help="JSON schedule the counters were taken with")
    args = ap.parse_args()
    if args.counters:
        summarize_counters(args.counters, args.record, args.record_workload,
                           json.loads(args.record_schedule) if args.record_schedule else None)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU (no collectives or sharding); "
                                   "use --gpus 1", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print(json.dumps({"error": "--steps must be >= 1 and --warmup >= 0"}))
        sys.exit(2)

    import torch
    import paper_1201_0499_amd as pe

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        copy_calibration(torch)
        return
    stream = torch.cuda.Stream()
    if args.only:
        run = {"paper_scale": lambda: measure_paper_scale(pe, torch, stream, args)[0],
               "newton": lambda: measure_newton(pe, torch, stream),
               "newton_large": lambda: measure_newton(pe, torch, stream, large=True),
               "track": lambda: measure_track(pe, torch, stream),
               "fp64_eval": lambda: measure_fp64_eval(pe, torch, stream),
               "batch": lambda: measure_batch(pe, torch, stream, args.tune_cache),
               "quad_double": lambda: measure_qd(pe, torch, stream)}[args.only]
        print(json.dumps({args.only: run()}))
        return

    head, side, big_sys, big_pts = measure_headline(pe, torch, stream, args)
    if not args.skip_side:
        ps, c2_sys, c2_pts, x, f, J = measure_paper_scale(pe, torch, stream, args)
        side["paper_scale"] = ps
        side["newton"] = measure_newton(pe, torch, stream)
        side["newton_large"] = measure_newton(pe, torch, stream, large=True)
        side["batch"] = measure_batch(pe, torch, stream, args.tune_cache)
        side["track"] = measure_track(pe, torch, stream)
        side["paper_layout"] = measure_paper_layout(pe, torch, stream, c2_sys, x, f, J,
                                                    ps["dd"]["us_per_evaluation"])
        side["quad_double"] = measure_qd(pe, torch, stream, c2_sys, c2_pts)

    cpu = None if args.no_cpu_baseline else measure_cpu(big_sys, big_pts, args.cpu_seconds)

    out = {
        "metric": "complex-dd monomial+gradient evals/s",
        "value": head["value"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (complex double-double)",
        "data": "synthetic (seeded random systems and unit-circle points of the stated shapes)",
        "config": head["config"],
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "paper_context": PAPER_C2050,
        "side": side,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
