"""Helpers shared by the GPU tests: device upload and the comparison metric.

The metric is a componentwise, condition-scaled error: for each output y,
|y_gpu - y_oracle| / S(y), where S(y) is the sum of magnitudes of the terms
that make up y (computed by the oracle).  Structural zeros (S = 0) must be
exactly zero on the GPU.
"""
import numpy as np
import torch

from oracle import ddoracle as O


def dev(planes):
    return tuple(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda() for a in planes)


def host(planes):
    return tuple(t.cpu().numpy() for t in planes)


def alloc(shape, n_planes=4):
    return tuple(torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
                 for _ in range(n_planes))


def scaled_err(got, ref, scale):
    """Max of |got - ref| / scale over entries with scale > 0, and whether
    every entry with scale == 0 is exactly zero in `got`."""
    d = O.dd_diff_abs(got, ref) if len(got) == 4 else np.hypot(got[0] - ref[0], got[1] - ref[1])
    pos = scale > 0
    err = float(np.max(d[pos] / scale[pos])) if np.any(pos) else 0.0
    zero_ok = True
    if np.any(~pos):
        for g in got:
            zero_ok &= bool(np.all(g[~pos] == 0.0))
    return err, zero_ok


def run_eval(system, pts, precision=1, with_jac=True, stream=None):
    """Evaluate through the C interface; returns host planes (f, J)."""
    import paper_1201_0499_amd as pe
    n, npoly = system.n_vars, system.n_polys
    P = pts[0].shape[0]
    x = dev(pts)
    f = alloc((P, npoly))
    J = alloc((P, n, npoly)) if with_jac else None
    if isinstance(system, pe.System):
        h = system.handle
    else:
        raise TypeError
    pe.eval_jac(h, P, x, f, J, precision, stream)
    torch.cuda.synchronize()
    return host(f), (host(J) if with_jac else None)
