"""Oracle: plain, slow FP64 CPU reference for the discrete eikonal system.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library never
links, imports or calls it, and it shares no code with the GPU library.

Functions (each cites the passage it follows; see ``eik_oracle.c``):

* ``godunov`` / ``godunov_f``  exact local solver of Eq 4 / Eq 6 (what
  Algorithms 1.1 and 1.3 compute), shifted form, float64 / float32.
* ``godunov_bisect``           the same root by bisection (independent check).
* ``fmm``      fast marching (Section 2.1) -- the plain definition of the result.
* ``fsm``      fast sweeping (Section 2.2), Gauss-Seidel to a fixed point.
* ``ifim``     Algorithm 2 emulated serially with synchronous reads, with the
               paper's per-phase work counters (float64 or float32 arithmetic).
* ``apply_local``  G_i(phi) for every node.
* ``adjoint``  dL/dF by a reverse sweep in fast-marching acceptance order.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eik_oracle.c")
_LIB = os.path.join(_HERE, "libeik_oracle.so")

EO_OK, EO_BAD, EO_NOCONV, EO_NOMEM = 0, 1, 2, 3
STAT_NAMES = ("step2_iters", "step3_iters", "evals_step2", "evals_detect",
              "evals_remedy", "remedy_initial", "max_active")


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no contraction, IEEE arithmetic)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        d, f, i, i64 = ctypes.c_double, ctypes.c_float, ctypes.c_int, ctypes.c_int64
        P = ctypes.c_void_p
        lib.eo_godunov.restype = d
        lib.eo_godunov.argtypes = [i, P, d]
        lib.eo_godunov_f.restype = f
        lib.eo_godunov_f.argtypes = [i, P, f]
        lib.eo_godunov_bisect.restype = d
        lib.eo_godunov_bisect.argtypes = [i, P, d]
        lib.eo_apply_local.restype = i
        lib.eo_apply_local.argtypes = [i, P, d, P, P, P]
        lib.eo_apply_local_f.restype = i
        lib.eo_apply_local_f.argtypes = [i, P, d, P, P, P]
        lib.eo_fmm.restype = i
        lib.eo_fmm.argtypes = [i, P, d, P, P, P, i64, P, P, P]
        lib.eo_fsm.restype = i
        lib.eo_fsm.argtypes = [i, P, d, P, P, P, i64, P, i, i64, P]
        lib.eo_ifim.restype = i
        lib.eo_ifim.argtypes = [i, P, d, P, P, P, i64, d, i, i64, P, P]
        lib.eo_ifim_f.restype = i
        lib.eo_ifim_f.argtypes = [i, P, d, P, P, P, i64, d, i, i64, P, P]
        lib.eo_fim.restype = i
        lib.eo_fim.argtypes = [i, P, d, P, P, P, i64, d, i64, P, P]
        # per-axis spacing variants (extra spacing pointer after h)
        lib.eo_godunov_aniso.restype = d
        lib.eo_godunov_aniso.argtypes = [i, P, P]
        lib.eo_godunov_aniso_f.restype = f
        lib.eo_godunov_aniso_f.argtypes = [i, P, P]
        lib.eo_apply_local_a.restype = i
        lib.eo_apply_local_a.argtypes = [i, P, d, P, P, P, P]
        lib.eo_apply_local_af.restype = i
        lib.eo_apply_local_af.argtypes = [i, P, P, P, P, P]
        lib.eo_fmm_a.restype = i
        lib.eo_fmm_a.argtypes = [i, P, d, P, P, P, P, i64, P, P, P]
        lib.eo_fsm_a.restype = i
        lib.eo_fsm_a.argtypes = [i, P, d, P, P, P, P, i64, P, i, i64, P]
        lib.eo_fim_a.restype = i
        lib.eo_fim_a.argtypes = [i, P, d, P, P, P, P, i64, d, i64, P, P]
        lib.eo_adjoint_a.restype = i
        lib.eo_adjoint_a.argtypes = [i, P, d, P, P, P, i64, P, P, P, P]
        if hasattr(lib, "eo_adjoint"):
            lib.eo_adjoint.restype = i
            lib.eo_adjoint.argtypes = [i, P, d, P, P, i64, P, P, P, P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _prep(F, sources, values):
    F64 = np.ascontiguousarray(np.asarray(F), dtype=np.float64)
    dims = np.asarray(F64.shape, dtype=np.int64)
    src = np.ascontiguousarray(np.asarray(sources, dtype=np.int64).ravel())
    val = None if values is None else np.ascontiguousarray(np.asarray(values, dtype=np.float64).ravel())
    if val is not None and val.shape != src.shape:
        raise ValueError("source values must match sources")
    return F64, dims, src, val


def godunov(a: Sequence[float], H: float) -> float:
    """Exact Godunov local solve from the per-axis minima `a` (Eq 4 / Eq 6)."""
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return float(_load().eo_godunov(len(arr), _ptr(arr), float(H)))


def godunov_f(a: Sequence[float], H: float) -> np.float32:
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    return np.float32(_load().eo_godunov_f(len(arr), _ptr(arr), float(np.float32(H))))


def godunov_bisect(a: Sequence[float], H: float) -> float:
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return float(_load().eo_godunov_bisect(len(arr), _ptr(arr), float(H)))


def _spacing(spacing, ndim):
    if spacing is None:
        return None
    sp = np.ascontiguousarray(np.asarray(spacing, dtype=np.float64).ravel())
    if sp.size != ndim or not np.all(np.isfinite(sp)) or not np.all(sp > 0):
        raise ValueError("spacing needs one finite positive entry per axis")
    return sp


def godunov_aniso(a: Sequence[float], H: Sequence[float], dtype=np.float64) -> float:
    """Local solve with a per-axis H_k = spacing_k / F (Eq 5 with dx != dy)."""
    if np.dtype(dtype) == np.float32:
        aa = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
        hh = np.ascontiguousarray(np.asarray(H, dtype=np.float32))
        return np.float32(_load().eo_godunov_aniso_f(len(aa), _ptr(aa), _ptr(hh)))
    aa = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    hh = np.ascontiguousarray(np.asarray(H, dtype=np.float64))
    return float(_load().eo_godunov_aniso(len(aa), _ptr(aa), _ptr(hh)))


def apply_local(F, h: float, phi, dtype=np.float64, spacing=None) -> np.ndarray:
    """G_i(phi) at every node, in float64 (default) or float32 arithmetic;
    spacing (one per axis, dims order) replaces the isotropic h."""
    sp = _spacing(spacing, np.ndim(F))
    if sp is not None:
        if np.dtype(dtype) == np.float32:
            F32 = np.ascontiguousarray(np.asarray(F), dtype=np.float32)
            p32 = np.ascontiguousarray(np.asarray(phi), dtype=np.float32)
            o32 = np.empty_like(F32)
            dims = np.asarray(F32.shape, dtype=np.int64)
            rc = _load().eo_apply_local_af(F32.ndim, _ptr(dims), _ptr(sp), _ptr(F32), _ptr(p32), _ptr(o32))
            if rc:
                raise ValueError("eo_apply_local_af failed: %d" % rc)
            return o32
        F64 = np.ascontiguousarray(np.asarray(F), dtype=np.float64)
        p = np.ascontiguousarray(np.asarray(phi), dtype=np.float64)
        out = np.empty_like(F64)
        dims = np.asarray(F64.shape, dtype=np.int64)
        rc = _load().eo_apply_local_a(F64.ndim, _ptr(dims), float(h), _ptr(sp), _ptr(F64), _ptr(p), _ptr(out))
        if rc:
            raise ValueError("eo_apply_local_a failed: %d" % rc)
        return out
    if np.dtype(dtype) == np.float32:
        F32 = np.ascontiguousarray(np.asarray(F), dtype=np.float32)
        p32 = np.ascontiguousarray(np.asarray(phi), dtype=np.float32)
        o32 = np.empty_like(F32)
        dims = np.asarray(F32.shape, dtype=np.int64)
        rc = _load().eo_apply_local_f(F32.ndim, _ptr(dims), float(h), _ptr(F32), _ptr(p32), _ptr(o32))
        if rc:
            raise ValueError("eo_apply_local_f failed: %d" % rc)
        return o32
    F64 = np.ascontiguousarray(np.asarray(F), dtype=np.float64)
    p = np.ascontiguousarray(np.asarray(phi), dtype=np.float64)
    out = np.empty_like(F64)
    dims = np.asarray(F64.shape, dtype=np.int64)
    rc = _load().eo_apply_local(F64.ndim, _ptr(dims), float(h), _ptr(F64), _ptr(p), _ptr(out))
    if rc:
        raise ValueError("eo_apply_local failed: %d" % rc)
    return out


def fmm(F, h: float, sources, values=None, return_order: bool = False, spacing=None):
    """Fast-marching solution (float64) of the discrete system; spacing (one
    per axis, dims order) replaces the isotropic h."""
    F64, dims, src, val = _prep(F, sources, values)
    sp = _spacing(spacing, F64.ndim)
    phi = np.empty_like(F64)
    order = np.empty(F64.size, dtype=np.int64) if return_order else None
    nacc = ctypes.c_int64(0)
    rc = _load().eo_fmm_a(F64.ndim, _ptr(dims), float(h), None if sp is None else _ptr(sp), _ptr(F64),
                          _ptr(src), None if val is None else _ptr(val), len(src), _ptr(phi),
                          None if order is None else _ptr(order), ctypes.byref(nacc))
    if rc:
        raise ValueError("eo_fmm failed: %d" % rc)
    if return_order:
        return phi, order[: nacc.value].copy()
    return phi


def fsm(F, h: float, sources, values=None, bisect: bool = False, max_passes: int = 100000, spacing=None):
    """Fast-sweeping (Gauss-Seidel) solution; returns (phi, passes)."""
    F64, dims, src, val = _prep(F, sources, values)
    sp = _spacing(spacing, F64.ndim)
    phi = np.empty_like(F64)
    passes = ctypes.c_int64(0)
    rc = _load().eo_fsm_a(F64.ndim, _ptr(dims), float(h), None if sp is None else _ptr(sp), _ptr(F64),
                          _ptr(src), None if val is None else _ptr(val), len(src), _ptr(phi),
                          1 if bisect else 0, int(max_passes), ctypes.byref(passes))
    if rc:
        raise ValueError("eo_fsm failed: %d" % rc)
    return phi, int(passes.value)


def ifim(F, h: float, sources, values=None, eps: float = 0.0, skip_remedy: bool = False,
         dtype=np.float64, max_iters: Optional[int] = None):
    """Algorithm 2 with synchronous reads; returns (phi, stats dict)."""
    F64, dims, src, val = _prep(F, sources, values)
    dt = np.dtype(dtype)
    phi = np.empty(F64.shape, dtype=dt)
    stats = np.zeros(len(STAT_NAMES), dtype=np.int64)
    cap = int(max_iters) if max_iters is not None else 4 * F64.size + 16
    fn = _load().eo_ifim if dt == np.float64 else _load().eo_ifim_f
    if dt not in (np.dtype(np.float64), np.dtype(np.float32)):
        raise ValueError("dtype must be float32 or float64")
    rc = fn(F64.ndim, _ptr(dims), float(h), _ptr(F64), _ptr(src),
            None if val is None else _ptr(val), len(src), float(eps),
            1 if skip_remedy else 0, cap, _ptr(phi), _ptr(stats))
    if rc == EO_NOCONV:
        raise RuntimeError("eo_ifim: iteration cap reached")
    if rc:
        raise ValueError("eo_ifim failed: %d" % rc)
    return phi, dict(zip(STAT_NAMES, (int(v) for v in stats)))


FIM_STAT_NAMES = ("iters", "evals_update", "evals_check", "max_active")


def fim(F, h: float, sources, values=None, eps: float = 0.0, max_iters: Optional[int] = None, spacing=None):
    """The fast iterative method (Section 2.3), serial, synchronous reads per
    iteration, float64; returns (phi, stats dict)."""
    F64, dims, src, val = _prep(F, sources, values)
    sp = _spacing(spacing, F64.ndim)
    phi = np.empty(F64.shape, dtype=np.float64)
    stats = np.zeros(len(FIM_STAT_NAMES), dtype=np.int64)
    cap = int(max_iters) if max_iters is not None else 4 * F64.size + 16
    rc = _load().eo_fim_a(F64.ndim, _ptr(dims), float(h), None if sp is None else _ptr(sp), _ptr(F64),
                          _ptr(src), None if val is None else _ptr(val), len(src), float(eps), cap, _ptr(phi),
                          _ptr(stats))
    if rc == EO_NOCONV:
        raise RuntimeError("eo_fim: iteration cap reached")
    if rc:
        raise ValueError("eo_fim failed: %d" % rc)
    return phi, dict(zip(FIM_STAT_NAMES, (int(v) for v in stats)))


def adjoint(F, h: float, sources, phi, dL_dphi, values=None, spacing=None, return_lambda: bool = False):
    """dL/dF for a loss L(phi), by reverse sweep in acceptance order (float64).
    With return_lambda, also the adjoint state lambda (lambda = dL/dphi +
    M^T lambda, the multiplier of each node's equation)."""
    lib = _load()
    if not hasattr(lib, "eo_adjoint"):
        raise NotImplementedError("oracle adjoint not built")
    F64, dims, src, val = _prep(F, sources, values)
    sp = _spacing(spacing, F64.ndim)
    p = np.ascontiguousarray(np.asarray(phi), dtype=np.float64)
    g = np.ascontiguousarray(np.asarray(dL_dphi), dtype=np.float64)
    out = np.empty_like(F64)
    lam = np.empty_like(F64) if return_lambda else None
    rc = lib.eo_adjoint_a(F64.ndim, _ptr(dims), float(h), None if sp is None else _ptr(sp), _ptr(F64),
                          _ptr(src), len(src), _ptr(p), _ptr(g), _ptr(out), None if lam is None else _ptr(lam))
    if rc:
        raise ValueError("eo_adjoint failed: %d" % rc)
    return (out, lam) if return_lambda else out
