"""The committed schedule cache of the autotuners and the keys bench.py
looks up in it (pure Python, no GPU).

The cache is a text file, one entry per line: a key naming the precision
and the shapes, then the tuned values (the last entry of a key wins).  A
system key is system-<dd|f64>:<n_vars>x<n_polys>x<n_monos>k<max k>d<max
exponent>p<points> with six values (lanes, chunk_vars, threads, groups,
tile_points, stage_buffers); a batch key is batch-<dd|f64> followed by one
:<n_vars>x<n_polys>x<n_monos>k<max k>d<max exponent>p<points> per system,
with four values (chunk_vars, threads, lanes multiple, task terms).
"""
import os

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNED = os.path.join(ROOT, "paper_1201_0499_amd", "tuned_schedules.txt")


def read_tuned(path=TUNED):
    out = {}
    if not os.path.exists(path):
        return out
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) >= 2:
                out[parts[0]] = [int(v) for v in parts[1:]]
    return out


def _shape(s, points):
    return f"{s.n_vars}x{s.n_polys}x{s.n_monos}k{s.max_k}d{s.max_exp}p{points}"


def system_key(s, points, dd):
    return f"system-{'dd' if dd else 'f64'}:{_shape(s, points)}"


def batch_key(systems, points, dd):
    return f"batch-{'dd' if dd else 'f64'}" + "".join(":" + _shape(s, p) for s, p in zip(systems, points))


def bench_system_keys():
    """Keys of the system schedules bench.py tunes: the large system at
    256 points and the paper-scale system at one point, in dd (1) and
    FP64 (0)."""
    big = synth.large_workload(n_points=1)[0]
    ps = synth.paper_scale_workload()[0]
    return {("large", 1): system_key(big, 256, True), ("large", 0): system_key(big, 256, False),
            ("paper_scale", 1): system_key(ps, 1, True),
            ("paper_scale", 0): system_key(ps, 1, False)}


def bench_batch_key():
    systems, pts = synth.batch_workload()
    return batch_key(systems, [p[0].shape[0] for p in pts], True)
