"""MI355X (gfx950) eikonal solver: the improved fast iterative method.

Thin Python binding of ``libeik.so`` (C ABI in ``include/eik.h``).  It only
marshals arguments: every step of a solve runs in the library's HIP kernels.
PyTorch provides device memory and the stream.  If the library is not built
the binding raises; there is no fallback path.

Functions mirror the C entry points:

* ``eik_solve``        Algorithm 2 (initialisation, update, remedy).
* ``eik_apply_local``  one dense pass of the exact Godunov local solve.
* ``eik_adjoint``      dL/dF at a converged solution.
* ``eik_solve_batch`` / ``eik_adjoint_batch``  the same for many grids at once.
* ``eik_async_status`` whether asynchronous (graph-captured) work converged.
* ``eik_solve_noalloc`` ``eik_solve`` on the library's static device scratch,
  allocating nothing (for callers that cannot allocate).
* ``eik_workspace_size``, ``eik_status_string``, ``eik_abi_version``.

``solve`` / ``apply_local`` / ``adjoint`` / ``solve_batch`` / ``adjoint_batch``
are the tensor-level wrappers and ``EikonalFn`` the autograd function built on
``eik_solve`` + ``eik_adjoint``.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple, Union

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libeik.so")

EIK_OK = 0
EIK_ERR_INVALID_ARGUMENT = 1
EIK_ERR_NO_CONVERGENCE = 2
EIK_ERR_OUT_OF_MEMORY = 3
EIK_ERR_DEVICE = 4
EIK_ERR_UNSUPPORTED = 5

EIK_FLOAT32 = 0
EIK_FLOAT64 = 1
EIK_VARIANT_NODE_LIST = 0
EIK_VARIANT_TILE = 1
EIK_VARIANT_FIM = 2
EIK_ABI_VERSION = 8
EIK_FLAG_DETERMINISTIC = 1
EIK_FLAG_SKIP_REMEDY = 2
EIK_FLAG_ASYNC = 4
EIK_FLAG_PROFILE = 8
EIK_FLAG_FIFO_REMEDY = 16
EIK_FLAG_NO_EARLY_REMEDY = 32

VARIANTS = {"node": EIK_VARIANT_NODE_LIST, "node_list": EIK_VARIANT_NODE_LIST,
            "tile": EIK_VARIANT_TILE, "fim": EIK_VARIANT_FIM}

# Entry points declared in include/eik.h
EXPORTS = ("eik_default_options", "eik_workspace_size", "eik_solve", "eik_apply_local",
           "eik_adjoint", "eik_adjoint_workspace_size", "eik_status_string", "eik_last_error",
           "eik_abi_version", "eik_solve_batch", "eik_batch_workspace_size", "eik_adjoint_batch",
           "eik_adjoint_batch_workspace_size", "eik_tune", "eik_async_status", "eik_solve_noalloc")


KERNEL_KINDS = ("update", "detect", "remedy", "adjoint", "other")


class EikInstance(ctypes.Structure):
    """eik_instance: one grid of a batch."""
    _fields_ = [("dims", ctypes.c_int64 * 3), ("h", ctypes.c_double), ("n_sources", ctypes.c_int64)]


class EikTuneEntry(ctypes.Structure):
    """eik_tune_entry: one timed candidate."""
    _fields_ = [("tile", ctypes.c_int32 * 3), ("inner_iters", ctypes.c_int32), ("ms", ctypes.c_double),
                ("order_min", ctypes.c_int32), ("workgroups", ctypes.c_int32)]


class EikStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "step2_iters", "step3_iters", "evals_step2", "evals_detect", "evals_remedy",
        "remedy_initial", "max_active", "launches", "tile_visits_step2", "tile_visits_step3",
        "inner_step2", "inner_step3", "written_step2", "written_step3", "evals_check",
        "evals_early")] + [
        ("kernel_launches", ctypes.c_int64 * 5), ("kernel_ms", ctypes.c_double * 5)]

    def to_dict(self):
        d = {n: int(getattr(self, n)) for n, t in self._fields_ if t is ctypes.c_int64}
        if any(self.kernel_launches):
            d["kernels"] = {k: {"launches": int(self.kernel_launches[i]), "ms": float(self.kernel_ms[i])}
                            for i, k in enumerate(KERNEL_KINDS)}
        return d


class EikOptions(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_int),
        ("variant", ctypes.c_int),
        ("tile", ctypes.c_int32 * 3),
        ("inner_iters", ctypes.c_int32),
        ("max_iters", ctypes.c_int64),
        ("flags", ctypes.c_uint32),
        ("source_values", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
        ("stats", ctypes.POINTER(EikStats)),
        ("spacing", ctypes.c_double * 3),
        ("order_min", ctypes.c_int32),
        ("workgroups", ctypes.c_int32),
    ]


class EikError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        super().__init__(f"{_status_name(status)}: {detail}")


_lib = None


def _status_name(s: int) -> str:
    try:
        return _load().eik_status_string(s).decode()
    except Exception:  # pragma: no cover
        return f"status {s}"


def _load():
    """Load libeik.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2106_15869_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    OP = ctypes.POINTER(EikOptions)
    lib.eik_default_options.restype = None
    lib.eik_default_options.argtypes = [OP]
    lib.eik_workspace_size.restype = ctypes.c_size_t
    lib.eik_workspace_size.argtypes = [i32, P, OP]
    lib.eik_solve.restype = ctypes.c_int
    lib.eik_solve.argtypes = [P, i32, P, d, P, i64, d, P, OP]
    lib.eik_apply_local.restype = ctypes.c_int
    lib.eik_apply_local.argtypes = [P, P, i32, P, d, P, OP]
    lib.eik_adjoint.restype = ctypes.c_int
    lib.eik_adjoint.argtypes = [P, P, i32, P, d, P, i64, P, P, OP]
    lib.eik_adjoint_workspace_size.restype = ctypes.c_size_t
    lib.eik_adjoint_workspace_size.argtypes = [i32, P, OP]
    lib.eik_status_string.restype = ctypes.c_char_p
    lib.eik_status_string.argtypes = [ctypes.c_int]
    lib.eik_last_error.restype = ctypes.c_char_p
    lib.eik_last_error.argtypes = []
    lib.eik_abi_version.restype = i32
    lib.eik_abi_version.argtypes = []
    lib.eik_tune.restype = ctypes.c_int
    lib.eik_tune.argtypes = [P, i32, P, d, P, i64, d, P, OP, ctypes.POINTER(EikTuneEntry), i32,
                             ctypes.POINTER(i32)]
    IP = ctypes.POINTER(EikInstance)
    lib.eik_solve_batch.restype = ctypes.c_int
    lib.eik_solve_batch.argtypes = [P, i32, IP, i32, P, d, P, OP]
    lib.eik_batch_workspace_size.restype = ctypes.c_size_t
    lib.eik_batch_workspace_size.argtypes = [i32, IP, i32, OP]
    lib.eik_adjoint_batch.restype = ctypes.c_int
    lib.eik_adjoint_batch.argtypes = [P, P, i32, IP, i32, P, P, P, OP]
    lib.eik_adjoint_batch_workspace_size.restype = ctypes.c_size_t
    lib.eik_adjoint_batch_workspace_size.argtypes = [i32, IP, i32, OP]
    lib.eik_async_status.restype = ctypes.c_int
    lib.eik_async_status.argtypes = [P, P]
    lib.eik_solve_noalloc.restype = ctypes.c_int
    lib.eik_solve_noalloc.argtypes = [P, i32, P, d, P, i64, d, P, OP]
    if lib.eik_abi_version() != EIK_ABI_VERSION:
        raise ImportError(f"{LIB_PATH} has ABI version {lib.eik_abi_version()}, this binding expects "
                          f"{EIK_ABI_VERSION}: rebuild it with `python -m paper_2106_15869_amd.build`")
    _lib = lib
    return lib


def lib():
    return _load()


def _check(rc: int):
    if rc != EIK_OK:
        raise EikError(rc, _load().eik_last_error().decode())


def make_options(dtype=None, variant: Union[str, int] = "tile", tile: Optional[Sequence[int]] = None,
                 inner_iters: int = 0, max_iters: int = 0, deterministic: bool = False,
                 skip_remedy: bool = False, async_: bool = False, profile: bool = False,
                 fifo: bool = False, spacing: Optional[Sequence[float]] = None, order_min: int = 0,
                 workgroups: int = 0, early: bool = True) -> EikOptions:
    o = EikOptions()
    _load().eik_default_options(ctypes.byref(o))
    if dtype is not None:
        o.dtype = dtype
    o.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    if tile is not None:
        t = list(tile)
        t = [0] * (3 - len(t)) + t if len(t) < 3 else t
        for k in range(3):
            o.tile[k] = int(t[k])
    o.inner_iters = int(inner_iters)
    o.max_iters = int(max_iters)
    o.flags = ((EIK_FLAG_DETERMINISTIC if deterministic else 0) |
               (EIK_FLAG_SKIP_REMEDY if skip_remedy else 0) |
               (EIK_FLAG_ASYNC if async_ else 0) |
               (EIK_FLAG_PROFILE if profile else 0) |
               (EIK_FLAG_FIFO_REMEDY if fifo else 0) |
               (0 if early else EIK_FLAG_NO_EARLY_REMEDY))
    if spacing is not None:
        for k, v in enumerate(spacing):
            o.spacing[k] = float(v)
    o.order_min = int(order_min)
    o.workgroups = int(workgroups)
    return o


def _dims(shape) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(list(shape), dtype=np.int64))


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def eik_workspace_size(shape: Sequence[int], opt: Optional[EikOptions] = None) -> int:
    dims = _dims(shape)
    return int(_load().eik_workspace_size(len(dims), _np_ptr(dims),
                                          ctypes.byref(opt) if opt is not None else None))


def eik_status_string(status: int) -> str:
    return _load().eik_status_string(status).decode()


def eik_abi_version() -> int:
    return int(_load().eik_abi_version())


def async_status(workspace, stream=None) -> int:
    """eik_async_status: outcome of the last asynchronous call (or graph
    replay) on `workspace` -- EIK_OK, EIK_ERR_NO_CONVERGENCE (a loop used up
    its launch budget) or EIK_ERR_INVALID_ARGUMENT (bad F).  Waits for the
    stream."""
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream(workspace.device)
    with torch.cuda.device(workspace.device):
        return int(_load().eik_async_status(workspace.data_ptr(), s.cuda_stream))


def check_async(workspace, stream=None) -> None:
    """Raise EikError unless the last asynchronous call on `workspace` converged."""
    _check(async_status(workspace, stream))


# ---------------------------------------------------------------------------
# tensor-level wrappers
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return EIK_FLOAT32
    if t.dtype == torch.float64:
        return EIK_FLOAT64
    raise TypeError("F must be float32 or float64")


def _check_device_tensor(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _sources_array(sources, shape) -> np.ndarray:
    arr = np.asarray(sources.cpu() if hasattr(sources, "cpu") else sources)
    if arr.ndim == 2 and arr.shape[1] == len(shape):
        arr = np.ravel_multi_index(tuple(arr.T.astype(np.int64)), tuple(shape))
    return np.ascontiguousarray(arr.astype(np.int64).ravel())


def solve(F, h: Optional[float], sources, eps: float = 0.0, *, variant: Union[str, int] = "tile",
          source_values=None, deterministic: bool = False, skip_remedy: bool = False,
          tile: Optional[Sequence[int]] = None, inner_iters: int = 0, max_iters: int = 0,
          out=None, workspace=None, stats: bool = False, stream=None, profile: bool = False,
          async_: bool = False, fifo: bool = False, spacing: Optional[Sequence[float]] = None,
          order_min: int = 0, workgroups: int = 0, early: bool = True):
    """Solve ||grad phi|| = 1/F on F's grid (2D or 3D device tensor).

    sources: flat indices, or an (n, ndim) array of coordinates.  Returns phi
    (and a stats dict when stats=True).  fifo=True runs the tile variant's
    remedy first-in first-out instead of in increasing pending value;
    early=False keeps the 3D tile variant's idle workgroups out of the update
    step (no early remedy visits).  async_=True only enqueues (no host
    synchronisation, capturable in a graph): it needs `workspace`, `out` and
    an explicit `max_iters`, and runs exactly max_iters launches per loop."""
    torch = _torch()
    _check_device_tensor(F, "F")
    if F.dim() not in (2, 3):
        raise ValueError("F must be 2D or 3D")
    opt = make_options(_dtype_code(F), variant, tile, inner_iters, max_iters, deterministic,
                       skip_remedy, async_=async_, profile=profile, fifo=fifo, spacing=spacing,
                       order_min=order_min, workgroups=workgroups, early=early)
    h = 1.0 if h is None and spacing is not None else h
    if async_ and (workspace is None or out is None):
        raise ValueError("async_ needs a preallocated workspace and out")
    dims = _dims(F.shape)
    src = _sources_array(sources, F.shape)
    vals = None
    if source_values is not None:
        vals = np.ascontiguousarray(np.asarray(source_values, dtype=np.float64).ravel())
        if vals.shape != src.shape:
            raise ValueError("source_values must match sources")
        opt.source_values = vals.ctypes.data
    phi = out if out is not None else torch.empty_like(F)
    _check_device_tensor(phi, "out")
    need = eik_workspace_size(F.shape, opt)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=F.device)
    elif workspace.numel() < need:
        raise ValueError(f"workspace needs {need} bytes")
    opt.workspace = workspace.data_ptr()
    opt.workspace_bytes = workspace.numel()
    st = EikStats()
    opt.stats = ctypes.pointer(st)
    s = stream if stream is not None else torch.cuda.current_stream(F.device)
    opt.stream = s.cuda_stream
    with torch.cuda.device(F.device):
        rc = _load().eik_solve(F.data_ptr(), F.dim(), _np_ptr(dims), float(h), _np_ptr(src),
                               len(src), float(eps), phi.data_ptr(), ctypes.byref(opt))
    _check(rc)
    return (phi, st.to_dict()) if stats else phi


def solve_noalloc(F, h: Optional[float], sources, eps: float = 0.0, *, out=None,
                  variant: Union[str, int] = "tile", source_values=None, deterministic: bool = False,
                  skip_remedy: bool = False, tile: Optional[Sequence[int]] = None, inner_iters: int = 0,
                  max_iters: int = 0, stats: bool = False, stream=None, fifo: bool = False,
                  spacing: Optional[Sequence[float]] = None, order_min: int = 0, workgroups: int = 0,
                  early: bool = True):
    """eik_solve_noalloc: solve() on the library's static device scratch (no
    workspace argument; the library allocates nothing).  Synchronous only.
    Pass `out` to keep the call free of allocations on this side too."""
    torch = _torch()
    _check_device_tensor(F, "F")
    if F.dim() not in (2, 3):
        raise ValueError("F must be 2D or 3D")
    opt = make_options(_dtype_code(F), variant, tile, inner_iters, max_iters, deterministic,
                       skip_remedy, fifo=fifo, spacing=spacing, order_min=order_min, workgroups=workgroups,
                       early=early)
    h = 1.0 if h is None and spacing is not None else h
    dims = _dims(F.shape)
    src = _sources_array(sources, F.shape)
    vals = None
    if source_values is not None:
        vals = np.ascontiguousarray(np.asarray(source_values, dtype=np.float64).ravel())
        if vals.shape != src.shape:
            raise ValueError("source_values must match sources")
        opt.source_values = vals.ctypes.data
    phi = out if out is not None else torch.empty_like(F)
    _check_device_tensor(phi, "out")
    if phi.shape != F.shape or phi.dtype != F.dtype:
        raise ValueError("out must match F in shape and dtype")
    st = EikStats()
    opt.stats = ctypes.pointer(st)
    s = stream if stream is not None else torch.cuda.current_stream(F.device)
    opt.stream = s.cuda_stream
    with torch.cuda.device(F.device):
        rc = _load().eik_solve_noalloc(F.data_ptr(), F.dim(), _np_ptr(dims), float(h), _np_ptr(src),
                                       len(src), float(eps), phi.data_ptr(), ctypes.byref(opt))
    _check(rc)
    return (phi, st.to_dict()) if stats else phi


def apply_local(F, phi, h: Optional[float], out=None, spacing: Optional[Sequence[float]] = None):
    """out_i = G_i(phi): the exact Godunov local solve at every node
    (spacing: one per axis for dx != dy; h may then be None)."""
    torch = _torch()
    _check_device_tensor(F, "F")
    _check_device_tensor(phi, "phi")
    if phi.shape != F.shape or phi.dtype != F.dtype:
        raise ValueError("phi must match F in shape and dtype")
    opt = make_options(_dtype_code(F), spacing=spacing)
    h = 1.0 if h is None and spacing is not None else h
    opt.stream = torch.cuda.current_stream(F.device).cuda_stream
    res = out if out is not None else torch.empty_like(F)
    dims = _dims(F.shape)
    with torch.cuda.device(F.device):
        rc = _load().eik_apply_local(F.data_ptr(), phi.data_ptr(), F.dim(), _np_ptr(dims), float(h),
                                     res.data_ptr(), ctypes.byref(opt))
    _check(rc)
    return res


def eik_adjoint_workspace_size(shape: Sequence[int], opt: Optional[EikOptions] = None) -> int:
    dims = _dims(shape)
    return int(_load().eik_adjoint_workspace_size(len(dims), _np_ptr(dims),
                                                  ctypes.byref(opt) if opt is not None else None))


def adjoint(F, phi, h: Optional[float], sources, dL_dphi, out=None, workspace=None, stats: bool = False,
            stream=None, profile: bool = False, async_: bool = False, max_iters: int = 0,
            spacing: Optional[Sequence[float]] = None, order_min: int = 0, workgroups: int = 0):
    """dL/dF at the converged solution phi (same F, h, sources).  async_,
    order_min and workgroups as in solve()."""
    torch = _torch()
    for t, n in ((F, "F"), (phi, "phi"), (dL_dphi, "dL_dphi")):
        _check_device_tensor(t, n)
        if t.shape != F.shape or t.dtype != F.dtype:
            raise ValueError(f"{n} must match F in shape and dtype")
    opt = make_options(_dtype_code(F), max_iters=max_iters, async_=async_, profile=profile, spacing=spacing,
                       order_min=order_min, workgroups=workgroups)
    h = 1.0 if h is None and spacing is not None else h
    if async_ and (workspace is None or out is None):
        raise ValueError("async_ needs a preallocated workspace and out")
    s = stream if stream is not None else torch.cuda.current_stream(F.device)
    opt.stream = s.cuda_stream
    need = eik_adjoint_workspace_size(F.shape, opt)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=F.device)
    elif workspace.numel() < need:
        raise ValueError(f"workspace needs {need} bytes")
    opt.workspace = workspace.data_ptr()
    opt.workspace_bytes = workspace.numel()
    st = EikStats()
    opt.stats = ctypes.pointer(st)
    res = out if out is not None else torch.empty_like(F)
    dims = _dims(F.shape)
    src = _sources_array(sources, F.shape)
    with torch.cuda.device(F.device):
        rc = _load().eik_adjoint(F.data_ptr(), phi.data_ptr(), F.dim(), _np_ptr(dims), float(h),
                                 _np_ptr(src), len(src), dL_dphi.data_ptr(), res.data_ptr(),
                                 ctypes.byref(opt))
    _check(rc)
    return (res, st.to_dict()) if stats else res


# ---------------------------------------------------------------------------
# batches: several independent grids solved together
# ---------------------------------------------------------------------------

def _instances(shapes, h, sources):
    shapes = [tuple(int(v) for v in sh) for sh in shapes]
    if not shapes:
        raise ValueError("need at least one grid")
    nd = len(shapes[0])
    if nd not in (2, 3) or any(len(sh) != nd for sh in shapes):
        raise ValueError("all grids must be 2D, or all 3D")
    hs = [float(h)] * len(shapes) if np.isscalar(h) else [float(v) for v in h]
    if len(hs) != len(shapes) or len(sources) != len(shapes):
        raise ValueError("h (if a list) and sources need one entry per grid")
    arr = (EikInstance * len(shapes))()
    src = []
    for k, sh in enumerate(shapes):
        sk = _sources_array(sources[k], sh)
        for j in range(nd):
            arr[k].dims[j] = sh[j]
        arr[k].h = hs[k]
        arr[k].n_sources = len(sk)
        src.append(sk)
    return nd, arr, np.ascontiguousarray(np.concatenate(src).astype(np.int64)), shapes


def batch_sizes(shapes) -> list:
    """Node count of every grid (offsets of the packed layout are their prefix sums)."""
    return [int(np.prod(sh)) for sh in shapes]


def pack(tensors):
    """Grids back to back in one flat device tensor (the batch layout)."""
    torch = _torch()
    return torch.cat([t.reshape(-1) for t in tensors])


def unpack(flat, shapes):
    """Views of the grids of a packed batch tensor."""
    out, o = [], 0
    for sh in shapes:
        n = int(np.prod(sh))
        out.append(flat[o:o + n].view(*sh))
        o += n
    return out


def eik_batch_workspace_size(shapes, h, sources, opt: Optional[EikOptions] = None) -> int:
    nd, arr, _, _ = _instances(shapes, h, sources)
    return int(_load().eik_batch_workspace_size(nd, arr, len(arr), ctypes.byref(opt) if opt is not None else None))


def solve_batch(F, shapes, h, sources, eps: float = 0.0, *, source_values=None,
                tile: Optional[Sequence[int]] = None, inner_iters: int = 0, max_iters: int = 0, out=None,
                workspace=None, stats: bool = False, stream=None, profile: bool = False, async_: bool = False,
                fifo: bool = False, order_min: int = 0, workgroups: int = 0, early: bool = True):
    """Solve several independent grids in one call (tile schedule).

    F: flat device tensor with the grids back to back (see pack()); shapes:
    one shape per grid; h: a spacing or one per grid; sources: per grid, flat
    indices local to that grid (or coordinate arrays).  Returns the packed phi
    (and summed stats)."""
    torch = _torch()
    _check_device_tensor(F, "F")
    nd, arr, src, shapes = _instances(shapes, h, sources)
    if F.numel() != sum(batch_sizes(shapes)):
        raise ValueError("F must hold exactly the grids of the batch")
    opt = make_options(_dtype_code(F), "tile", tile, inner_iters, max_iters, async_=async_, profile=profile,
                       fifo=fifo, order_min=order_min, workgroups=workgroups, early=early)
    if async_ and (workspace is None or out is None):
        raise ValueError("async_ needs a preallocated workspace and out")
    vals = None
    if source_values is not None:
        vals = np.ascontiguousarray(np.concatenate([np.asarray(v, dtype=np.float64).ravel()
                                                    for v in source_values]))
        if vals.shape != src.shape:
            raise ValueError("source_values must match sources")
        opt.source_values = vals.ctypes.data
    phi = out if out is not None else torch.empty_like(F)
    _check_device_tensor(phi, "out")
    need = int(_load().eik_batch_workspace_size(nd, arr, len(arr), ctypes.byref(opt)))
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=F.device)
    elif workspace.numel() < need:
        raise ValueError(f"workspace needs {need} bytes")
    opt.workspace = workspace.data_ptr()
    opt.workspace_bytes = workspace.numel()
    st = EikStats()
    opt.stats = ctypes.pointer(st)
    s = stream if stream is not None else torch.cuda.current_stream(F.device)
    opt.stream = s.cuda_stream
    with torch.cuda.device(F.device):
        rc = _load().eik_solve_batch(F.data_ptr(), nd, arr, len(arr), _np_ptr(src), float(eps), phi.data_ptr(),
                                     ctypes.byref(opt))
    _check(rc)
    return (phi, st.to_dict()) if stats else phi


def eik_adjoint_batch_workspace_size(shapes, h, sources, opt: Optional[EikOptions] = None) -> int:
    nd, arr, _, _ = _instances(shapes, h, sources)
    return int(_load().eik_adjoint_batch_workspace_size(nd, arr, len(arr),
                                                        ctypes.byref(opt) if opt is not None else None))


def adjoint_batch(F, phi, shapes, h, sources, dL_dphi, *, out=None, workspace=None, stats: bool = False,
                  stream=None, profile: bool = False, async_: bool = False, max_iters: int = 0):
    """dL/dF for every grid of a batch (packed layout as solve_batch)."""
    torch = _torch()
    for t, n in ((F, "F"), (phi, "phi"), (dL_dphi, "dL_dphi")):
        _check_device_tensor(t, n)
        if t.shape != F.shape or t.dtype != F.dtype:
            raise ValueError(f"{n} must match F in shape and dtype")
    nd, arr, src, shapes = _instances(shapes, h, sources)
    if F.numel() != sum(batch_sizes(shapes)):
        raise ValueError("F must hold exactly the grids of the batch")
    opt = make_options(_dtype_code(F), max_iters=max_iters, async_=async_, profile=profile)
    if async_ and (workspace is None or out is None):
        raise ValueError("async_ needs a preallocated workspace and out")
    need = int(_load().eik_adjoint_batch_workspace_size(nd, arr, len(arr), ctypes.byref(opt)))
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=F.device)
    elif workspace.numel() < need:
        raise ValueError(f"workspace needs {need} bytes")
    opt.workspace = workspace.data_ptr()
    opt.workspace_bytes = workspace.numel()
    st = EikStats()
    opt.stats = ctypes.pointer(st)
    s = stream if stream is not None else torch.cuda.current_stream(F.device)
    opt.stream = s.cuda_stream
    res = out if out is not None else torch.empty_like(F)
    with torch.cuda.device(F.device):
        rc = _load().eik_adjoint_batch(F.data_ptr(), phi.data_ptr(), nd, arr, len(arr), _np_ptr(src),
                                       dL_dphi.data_ptr(), res.data_ptr(), ctypes.byref(opt))
    _check(rc)
    return (res, st.to_dict()) if stats else res


def tune(F, h: Optional[float], sources, eps: float = 0.0, *, stream=None, workspace=None,
         spacing: Optional[Sequence[float]] = None, fifo: bool = False):
    """Time the tile-variant candidates on this problem (eik_tune) and return
    {"tile": (z, y, x), "inner_iters": k, "order_min": m, "workgroups": w,
    "candidates": [...]} -- pass them to solve().  Cached per (ndim, dtype, log2 N, per-axis spacing
    or not, remedy schedule) for the process; a cached answer reports no
    candidates.  fifo: tune the first-in first-out remedy schedule."""
    torch = _torch()
    _check_device_tensor(F, "F")
    opt = make_options(_dtype_code(F), spacing=spacing, fifo=fifo)
    h = 1.0 if h is None and spacing is not None else h
    s = stream if stream is not None else torch.cuda.current_stream(F.device)
    opt.stream = s.cuda_stream
    if workspace is not None:
        opt.workspace = workspace.data_ptr()
        opt.workspace_bytes = workspace.numel()
    dims = _dims(F.shape)
    src = _sources_array(sources, F.shape)
    scratch = torch.empty_like(F)
    rep = (EikTuneEntry * 16)()
    nrep = ctypes.c_int32(0)
    with torch.cuda.device(F.device):
        rc = _load().eik_tune(F.data_ptr(), F.dim(), _np_ptr(dims), float(h), _np_ptr(src), len(src), float(eps),
                              scratch.data_ptr(), ctypes.byref(opt), rep, 16, ctypes.byref(nrep))
    _check(rc)
    cands = [{"tile": tuple(int(v) for v in rep[k].tile), "inner_iters": int(rep[k].inner_iters),
              "order_min": int(rep[k].order_min), "workgroups": int(rep[k].workgroups),
              "ms": float(rep[k].ms)} for k in range(nrep.value)]
    return {"tile": tuple(int(v) for v in opt.tile), "inner_iters": int(opt.inner_iters),
            "order_min": int(opt.order_min), "workgroups": int(opt.workgroups), "candidates": cands}


def _make_eikonal_fn():
    torch = _torch()

    class EikonalFn(torch.autograd.Function):
        """phi = EikonalFn.apply(F, h, sources[, variant]) with dL/dF from eik_adjoint."""

        @staticmethod
        def forward(ctx, F, h, sources, variant="tile"):
            Fc = F.detach().contiguous()
            phi = solve(Fc, h, sources, variant=variant)
            ctx.save_for_backward(Fc, phi)
            ctx.h = float(h)
            ctx.sources = _sources_array(sources, F.shape)
            return phi

        @staticmethod
        def backward(ctx, grad_phi):
            Fc, phi = ctx.saved_tensors
            g = grad_phi.contiguous()
            # unreached nodes carry no gradient (their phi is +inf)
            g = torch.where(torch.isfinite(phi), g, torch.zeros_like(g))
            dF = adjoint(Fc, phi, ctx.h, ctx.sources, g)
            return dF, None, None, None

    return EikonalFn


_EikonalFn = None


def __getattr__(name):
    global _EikonalFn
    if name == "EikonalFn":
        if _EikonalFn is None:
            _EikonalFn = _make_eikonal_fn()
        return _EikonalFn
    raise AttributeError(name)
