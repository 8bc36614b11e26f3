"""ORACLE -- test infrastructure only.

A plain CPU path tracker for the total-degree homotopy

    H(x, t) = (1 - t) gamma G(x) + t F(x),   G_i(x) = x_i^{d_i} - 1,

d_i the total degree of f_i: root finding by continuation, the use the
paper's introduction names for fast evaluation and Newton's method
(Section 1).  One path at a time, in numpy complex128, with F and its
Jacobian from the definitional evaluator of ``ddoracle`` (Section 2,
equation (1)).  The rules are those the library documents for pe_track:

- predictor: Euler step along the tangent, dx/dt = -H_x^{-1} H_t with
  H_x = t J_F + (1 - t) gamma diag(d_i x_i^{d_i - 1}) and H_t = F - gamma G,
  of length h clipped to 1 - t;
- corrector: up to ``corr_iters`` Newton steps on H(., t + h); converged when
  the last step has max |dx_i| <= corr_tol (1 + max |x_i|);
- step control: an accepted step doubles h (up to h_max) after three
  accepted steps in a row; a rejected one returns to the last accepted
  point with h halved, and the path stops when h < h_min;
- statuses: 0 reached t = 1, 1 step below h_min, 2 singular H_x,
  3 non-finite values, 4 step limit, 5 endgame failed;
- endgame: the oracle's plain dd Newton at t = 1.

It shares no code with the GPU library and the library never imports it.
"""
from __future__ import annotations

import numpy as np

from . import ddoracle as O


def total_degrees(system) -> np.ndarray:
    """Largest sum of exponents over the monomials of each polynomial."""
    deg = np.zeros(system.n_polys, np.int64)
    for p in range(system.n_polys):
        for s in range(int(system.poly_start[p]), int(system.poly_start[p + 1])):
            a, b = int(system.mono_start[s]), int(system.mono_start[s + 1])
            deg[p] = max(deg[p], int(np.sum(system.exp[a:b])))
    return deg


def start_solutions(system, first: int, n_paths: int) -> np.ndarray:
    """Start solutions first .. first+n_paths-1 of G (complex [P][n]): path q
    has mixed-radix digits k_i in base d_i, the digit of x_0 varying
    fastest, and x_i = exp(2 pi i k_i / d_i)."""
    d = total_degrees(system)
    out = np.empty((n_paths, system.n_vars), np.complex128)
    for p in range(n_paths):
        q = first + p
        for i in range(system.n_vars):
            k = q % int(d[i])
            q //= int(d[i])
            out[p, i] = np.exp(2j * np.pi * k / d[i])
    return out


def _FJ(system, x):
    (fr, fi), (Jr, Ji) = O.eval_f64(system, x.real[None, :].copy(), x.imag[None, :].copy())
    F = fr[0] + 1j * fi[0]
    # J[i][p] = df_p / dx_i  ->  A[p][i]
    A = (Jr[0] + 1j * Ji[0]).T
    return F, A


def _pieces(system, x, t, gamma, d):
    F, JF = _FJ(system, x)
    G = x ** d - 1.0
    Hx = t * JF + np.diag((1.0 - t) * gamma * d * x ** (d - 1))
    return F, G, Hx


def _solve(A, b):
    try:
        return np.linalg.solve(A, b)
    except np.linalg.LinAlgError:
        return None


def track_path(system, x0, gamma=0.6 + 0.8j, h_init=0.02, h_min=1e-10, h_max=0.1,
               corr_tol=1e-10, corr_iters=4, max_steps=4000):
    """Track one path from x0 (complex [n]) at t = 0.
    Returns (x, t, steps, status)."""
    d = total_degrees(system).astype(np.float64)
    xs = np.array(x0, dtype=np.complex128)
    t, h, succ, steps = 0.0, float(h_init), 0, 0
    while True:
        if steps >= max_steps:
            return xs, t, steps, 4
        F, G, Hx = _pieces(system, xs, t, gamma, d)
        v = _solve(Hx, F - gamma * G)
        if v is None:
            return xs, t, steps, 2
        hh = min(h, 1.0 - t)
        t1 = 1.0 if hh >= 1.0 - t else t + hh
        x = xs - hh * v
        steps += 1
        if not np.all(np.isfinite(x)):
            return xs, t, steps, 3
        accepted = False
        for _ in range(corr_iters):
            F, G, Hx = _pieces(system, x, t1, gamma, d)
            dx = _solve(Hx, t1 * F + (1.0 - t1) * gamma * G)
            if dx is None:
                return xs, t, steps, 2
            x = x - dx
            if not np.all(np.isfinite(x)):
                return xs, t, steps, 3
            if np.max(np.abs(dx)) <= corr_tol * (1.0 + np.max(np.abs(x))):
                accepted = True
                break
        if accepted:
            t, xs = t1, x
            succ += 1
            if succ >= 3:
                h, succ = min(2.0 * h, h_max), 0
            if t >= 1.0:
                return xs, t, steps, 0
        else:
            h, succ = 0.5 * h, 0
            if h < h_min:
                return xs, t, steps, 1


def track(system, x0, end_tol=1e-28, end_iters=8, **params):
    """Track every row of x0 (complex [P][n]); then, for the paths that
    reached t = 1, the dd Newton endgame (if end_tol > 0).  Returns
    (x_planes dd [4][P][n], t, steps, status, res)."""
    x0 = np.atleast_2d(np.asarray(x0, np.complex128))
    P, n = x0.shape
    X = np.empty_like(x0)
    T = np.zeros(P)
    steps = np.zeros(P, np.int64)
    status = np.zeros(P, np.int64)
    for p in range(P):
        X[p], T[p], steps[p], status[p] = track_path(system, x0[p], **params)
    planes = [X.real.copy(), np.zeros((P, n)), X.imag.copy(), np.zeros((P, n))]
    res = np.full(P, np.nan)
    if end_tol > 0:
        done = np.nonzero(status == 0)[0]
        if done.size:
            sub = [a[done] for a in planes]
            xr, r, _, st = O.newton_dd(system, sub, tol=end_tol, max_iter=end_iters)
            for q in range(4):
                planes[q][done] = xr[q]
            res[done] = r
            status[done[st != 0]] = 5
    return planes, T, steps, status, res
