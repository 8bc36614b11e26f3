"""polyeval on MI355X: Python binding of ``libpolyeval.so``.

Thin ctypes marshalling over the C interface declared in
``include/polyeval.h``; every step of the evaluation runs in the library's
HIP kernels.  PyTorch is used only to hold device memory and to name the
current HIP stream.  The binding fails loudly if the library is missing:
there is no fallback.

Complex arrays are passed as tuples of four float64 tensors
``(re_hi, re_lo, im_hi, im_lo)`` (double-double) -- in FP64 mode the two
``lo`` entries may be ``None``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from ._abi import (PE_DD, PE_FP64, PE_NEWTON_DD, PE_NEWTON_MIXED, PolyevalError, cvec,
                   check, lib, LIB_PATH,
                   pe_track_params)

__all__ = [
    "PE_DD", "PE_FP64", "PE_NEWTON_MIXED", "PE_NEWTON_DD", "PolyevalError", "lib", "LIB_PATH",
    "create_system", "destroy_system", "system_info", "eval_jac", "eval_jac_noalloc", "set_schedule",
    "get_schedule", "newton", "autotune_system", "System", "Batch",
]


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def create_system(n_vars, n_polys, poly_start, mono_start, pos, exp, coef):
    """``pe_create_system``: returns an opaque handle (int).  ``coef`` is a
    4-tuple of host float64 arrays."""
    ps, ms, ps_, ex = _i64(poly_start), _i64(mono_start), _i32(pos), _i32(exp)
    cs = [_f64(c) for c in coef]
    n_monos = ms.size - 1
    h = C.c_void_p()
    check(lib().pe_create_system(
        int(n_vars), int(n_polys), int(n_monos),
        ps.ctypes.data_as(C.POINTER(C.c_int64)), ms.ctypes.data_as(C.POINTER(C.c_int64)),
        ps_.ctypes.data_as(C.POINTER(C.c_int32)), ex.ctypes.data_as(C.POINTER(C.c_int32)),
        cvec([c.ctypes.data for c in cs]), C.byref(h)), "pe_create_system")
    return h.value


def destroy_system(handle):
    check(lib().pe_destroy_system(C.c_void_p(handle)), "pe_destroy_system")


def system_info(handle):
    nv, npl, mk, me = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    nm = C.c_int64()
    check(lib().pe_system_info(C.c_void_p(handle), C.byref(nv), C.byref(npl), C.byref(nm),
                               C.byref(mk), C.byref(me)), "pe_system_info")
    return dict(n_vars=nv.value, n_polys=npl.value, n_monos=nm.value, max_k=mk.value,
                max_exp=me.value)


def _dev_planes(planes, required_lo: bool):
    if planes is None:
        return cvec([0, 0, 0, 0])
    ptrs = []
    for j, t in enumerate(planes):
        if t is None:
            if required_lo or j in (0, 2):
                raise ValueError("missing plane")
            ptrs.append(0)
            continue
        if not t.is_cuda or t.dtype.__str__() != "torch.float64" or not t.is_contiguous():
            raise ValueError("planes must be contiguous float64 CUDA tensors")
        ptrs.append(t.data_ptr())
    return cvec(ptrs)


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


def eval_jac(handle, n_points, points, out_f, out_J=None, precision=PE_DD, stream=None):
    """``pe_eval_jac`` on device tensors: points ``[P][n]``, out_f
    ``[P][n_polys]``, out_J ``[P][n][n_polys]`` (or None)."""
    dd = precision == PE_DD
    check(lib().pe_eval_jac(C.c_void_p(handle), int(n_points), _dev_planes(points, dd),
                            _dev_planes(out_f, dd), _dev_planes(out_J, dd), int(precision),
                            C.c_void_p(_stream(stream))), "pe_eval_jac")


def eval_jac_noalloc(handle, n_points, points, out_f, out_J=None, precision=PE_DD, stream=None):
    """``pe_eval_jac_noalloc``: as eval_jac, allocating nothing (the schedule's
    tables must exist: call eval_jac once with n_points first)."""
    dd = precision == PE_DD
    check(lib().pe_eval_jac_noalloc(C.c_void_p(handle), int(n_points), _dev_planes(points, dd),
                                    _dev_planes(out_f, dd), _dev_planes(out_J, dd), int(precision),
                                    C.c_void_p(_stream(stream))), "pe_eval_jac_noalloc")


def _plane8(tensors):
    if tensors is None:
        return None
    if len(tensors) != 8:
        raise ValueError("quad-double values need 8 planes")
    arr = (C.c_void_p * 8)(*[C.c_void_p(t.data_ptr()) for t in tensors])
    return C.cast(arr, C.POINTER(C.c_void_p)), arr


def eval_jac_qd(handle, n_points, points, out_f, out_J=None, stream=None):
    """``pe_eval_jac_qd``: points, out_f and out_J (or None) are 8 device
    tensors each (re x0..x3, im x0..x3)."""
    p, keep_p = _plane8(points)
    f, keep_f = _plane8(out_f)
    J = _plane8(out_J)
    check(lib().pe_eval_jac_qd(C.c_void_p(handle), int(n_points), p, f, J[0] if J else None,
                               C.c_void_p(_stream(stream))), "pe_eval_jac_qd")


def eval_jac_paper_layout(handle, n_points, points, out_f, out_J=None, precision=PE_DD,
                          stream=None):
    """``pe_eval_jac_paper_layout``: the paper's three-kernel evaluation,
    same tensors as eval_jac."""
    dd = precision == PE_DD
    check(lib().pe_eval_jac_paper_layout(C.c_void_p(handle), int(n_points), _dev_planes(points, dd),
                                         _dev_planes(out_f, dd), _dev_planes(out_J, dd),
                                         int(precision), C.c_void_p(_stream(stream))),
          "pe_eval_jac_paper_layout")


def set_schedule(handle, lanes=0, chunk_vars=0, threads=0, groups=0, tile_points=0,
                 stage_buffers=0):
    check(lib().pe_set_schedule(C.c_void_p(handle), int(lanes), int(chunk_vars), int(threads),
                                int(groups), int(tile_points), int(stage_buffers)),
          "pe_set_schedule")


def get_schedule(handle, n_points):
    v = [C.c_int32() for _ in range(6)]
    check(lib().pe_get_schedule(C.c_void_p(handle), int(n_points), *[C.byref(x) for x in v]),
          "pe_get_schedule")
    return dict(lanes=v[0].value, chunk_vars=v[1].value, threads=v[2].value, groups=v[3].value,
                tile_points=v[4].value, stage_buffers=v[5].value)


def newton(handle, n_starts, x, res, iters, status, tol=1e-28, max_iter=10,
           mode=PE_NEWTON_MIXED, stream=None):
    """``pe_newton``: x (4 dd planes, device, updated in place), res (float64),
    iters and status (int32) device tensors of length n_starts.  Returns the
    status code (0 = all converged, 5 = some did not); raises on errors."""
    st = lib().pe_newton(C.c_void_p(handle), int(n_starts), _dev_planes(x, True), float(tol),
                         int(max_iter), int(mode), C.c_void_p(res.data_ptr()),
                         C.c_void_p(iters.data_ptr()), C.c_void_p(status.data_ptr()),
                         C.c_void_p(_stream(stream)))
    if st not in (0, 5):
        check(st, "pe_newton")
    return st


def newton_qd(handle, n_starts, x, res, iters, status, tol=1e-56, max_iter=10, stream=None):
    """``pe_newton_qd``: x (8 quad-double planes, device, updated in place),
    res (float64), iters and status (int32) device tensors of length
    n_starts.  Returns the status code (0 = all converged, 5 = some did
    not); raises on errors."""
    xp, keep = _plane8(x)
    st = lib().pe_newton_qd(C.c_void_p(handle), int(n_starts), xp, float(tol), int(max_iter),
                            C.c_void_p(res.data_ptr()), C.c_void_p(iters.data_ptr()),
                            C.c_void_p(status.data_ptr()), C.c_void_p(_stream(stream)))
    if st not in (0, 5):
        check(st, "pe_newton_qd")
    return st


TRACK_DEFAULTS = dict(gamma=complex(0.6, 0.8), h_init=0.02, h_min=1e-10, h_max=0.1,
                      corr_tol=1e-10, corr_iters=4, max_steps=4000, end_tol=1e-28, end_iters=8)


def start_solutions(handle, first, n_paths, x, stream=None):
    """``pe_start_solutions``: x (4 dd planes, device) <- start solutions
    first .. first+n_paths-1 of the total-degree start system."""
    check(lib().pe_start_solutions(C.c_void_p(handle), int(first), int(n_paths),
                                   _dev_planes(x, True), C.c_void_p(_stream(stream))),
          "pe_start_solutions")


def track(handle, n_paths, x, t, steps, status, res, stream=None, **params):
    """``pe_track``: x (4 dd planes, device, start solutions in, end points
    out), t and res (float64), steps and status (int32) device tensors of
    length n_paths.  Keyword parameters override TRACK_DEFAULTS.  Returns the
    status code (0 = every path reached a root, 5 = some did not)."""
    p = dict(TRACK_DEFAULTS)
    unknown = set(params) - set(p)
    if unknown:
        raise TypeError(f"unknown tracker parameters {sorted(unknown)}")
    p.update(params)
    g = complex(p["gamma"])
    prm = pe_track_params(g.real, g.imag, float(p["h_init"]), float(p["h_min"]), float(p["h_max"]),
                          float(p["corr_tol"]), int(p["corr_iters"]), int(p["max_steps"]),
                          float(p["end_tol"]), int(p["end_iters"]))
    st = lib().pe_track(C.c_void_p(handle), int(n_paths), _dev_planes(x, True), C.byref(prm),
                        C.c_void_p(t.data_ptr()), C.c_void_p(steps.data_ptr()),
                        C.c_void_p(status.data_ptr()), C.c_void_p(res.data_ptr()),
                        C.c_void_p(_stream(stream)))
    if st not in (0, 5):
        check(st, "pe_track")
    return st


def autotune_system(handle, n_points, points, out_f, out_J=None, precision=PE_DD, stream=None,
                    cache_path=None):
    """``pe_autotune_system``: time schedules on these buffers, pin the best."""
    dd = precision == PE_DD
    check(lib().pe_autotune_system(C.c_void_p(handle), int(n_points), _dev_planes(points, dd),
                                   _dev_planes(out_f, dd), _dev_planes(out_J, dd), int(precision),
                                   C.c_void_p(_stream(stream)),
                                   cache_path.encode() if cache_path else None),
          "pe_autotune_system")


class Batch:
    """Owning wrapper around a ``pe_batch`` over ``System`` objects (which
    must stay alive as long as the batch)."""

    def __init__(self, systems):
        self.systems = list(systems)
        arr = (C.c_void_p * len(self.systems))(*[s.handle for s in self.systems])
        h = C.c_void_p()
        check(lib().pe_create_batch(arr, len(self.systems), C.byref(h)), "pe_create_batch")
        self.handle = h.value

    def layout(self, points_per_system):
        pps = _i64(points_per_system)
        n = len(self.systems) + 1
        xo, fo, jo = (np.zeros(n, np.int64) for _ in range(3))
        P = C.POINTER(C.c_int64)
        check(lib().pe_batch_layout(C.c_void_p(self.handle), pps.ctypes.data_as(P),
                                    xo.ctypes.data_as(P), fo.ctypes.data_as(P),
                                    jo.ctypes.data_as(P)), "pe_batch_layout")
        return xo, fo, jo

    def eval_jac(self, points_per_system, points, out_f, out_J=None, precision=PE_DD, stream=None):
        dd = precision == PE_DD
        pps = _i64(points_per_system)
        check(lib().pe_eval_jac_batch(C.c_void_p(self.handle),
                                      pps.ctypes.data_as(C.POINTER(C.c_int64)),
                                      _dev_planes(points, dd), _dev_planes(out_f, dd),
                                      _dev_planes(out_J, dd), int(precision),
                                      C.c_void_p(_stream(stream))), "pe_eval_jac_batch")

    def autotune(self, points_per_system, points, out_f, out_J=None, precision=PE_DD, stream=None,
                 cache_path=None):
        dd = precision == PE_DD
        pps = _i64(points_per_system)
        check(lib().pe_autotune_batch(C.c_void_p(self.handle),
                                      pps.ctypes.data_as(C.POINTER(C.c_int64)),
                                      _dev_planes(points, dd), _dev_planes(out_f, dd),
                                      _dev_planes(out_J, dd), int(precision),
                                      C.c_void_p(_stream(stream)),
                                      cache_path.encode() if cache_path else None),
              "pe_autotune_batch")

    def config(self):
        v = [C.c_int32() for _ in range(4)]
        check(lib().pe_batch_config(C.c_void_p(self.handle), *[C.byref(x) for x in v]),
              "pe_batch_config")
        return dict(chunk_vars=v[0].value, threads=v[1].value, lanes_mult=v[2].value,
                    task_terms=v[3].value)

    def close(self):
        if getattr(self, "handle", None):
            lib().pe_destroy_batch(C.c_void_p(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class System:
    """Owning wrapper around a ``pe_system`` handle."""

    def __init__(self, n_vars, n_polys, poly_start, mono_start, pos, exp, coef):
        self.n_vars, self.n_polys = int(n_vars), int(n_polys)
        self.handle = create_system(n_vars, n_polys, poly_start, mono_start, pos, exp, coef)

    @classmethod
    def from_csr(cls, s):
        """From any object with n_vars, n_polys, poly_start, mono_start, pos,
        exp and coef (4 planes) attributes."""
        return cls(s.n_vars, s.n_polys, s.poly_start, s.mono_start, s.pos, s.exp, s.coef)

    def info(self):
        return system_info(self.handle)

    def eval_jac(self, n_points, points, out_f, out_J=None, precision=PE_DD, stream=None):
        eval_jac(self.handle, n_points, points, out_f, out_J, precision, stream)

    def eval_jac_noalloc(self, n_points, points, out_f, out_J=None, precision=PE_DD, stream=None):
        eval_jac_noalloc(self.handle, n_points, points, out_f, out_J, precision, stream)

    def eval_jac_qd(self, n_points, points, out_f, out_J=None, stream=None):
        eval_jac_qd(self.handle, n_points, points, out_f, out_J, stream)

    def eval_jac_paper_layout(self, n_points, points, out_f, out_J=None, precision=PE_DD,
                              stream=None):
        eval_jac_paper_layout(self.handle, n_points, points, out_f, out_J, precision, stream)

    def set_schedule(self, lanes=0, chunk_vars=0, threads=0, groups=0, tile_points=0,
                     stage_buffers=0):
        set_schedule(self.handle, lanes, chunk_vars, threads, groups, tile_points, stage_buffers)

    def get_schedule(self, n_points):
        return get_schedule(self.handle, n_points)

    def newton(self, n_starts, x, res, iters, status, tol=1e-28, max_iter=10,
               mode=PE_NEWTON_MIXED, stream=None):
        return newton(self.handle, n_starts, x, res, iters, status, tol, max_iter, mode, stream)

    def newton_qd(self, n_starts, x, res, iters, status, tol=1e-56, max_iter=10, stream=None):
        return newton_qd(self.handle, n_starts, x, res, iters, status, tol, max_iter, stream)

    def autotune(self, n_points, points, out_f, out_J=None, precision=PE_DD, stream=None,
                 cache_path=None):
        autotune_system(self.handle, n_points, points, out_f, out_J, precision, stream, cache_path)

    def start_solutions(self, first, n_paths, x, stream=None):
        start_solutions(self.handle, first, n_paths, x, stream)

    def track(self, n_paths, x, t, steps, status, res, stream=None, **params):
        return track(self.handle, n_paths, x, t, steps, status, res, stream, **params)

    def close(self):
        if getattr(self, "handle", None):
            destroy_system(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
