"""Independent checks of an eikonal solution, written from the defining
equations rather than from any solver (Eq 4 / Eq 6 and their consequences)."""

from __future__ import annotations

import numpy as np


def axis_minima(phi: np.ndarray) -> np.ndarray:
    """a_k = min(phi[i - e_k], phi[i + e_k]) per axis, +inf outside the grid."""
    phi = np.asarray(phi, dtype=np.float64)
    out = np.empty((phi.ndim,) + phi.shape, dtype=np.float64)
    for k in range(phi.ndim):
        pad = [(0, 0)] * phi.ndim
        pad[k] = (1, 1)
        p = np.pad(phi, pad, constant_values=np.inf)
        lo = [slice(None)] * phi.ndim
        hi = [slice(None)] * phi.ndim
        lo[k] = slice(0, -2)
        hi[k] = slice(2, None)
        out[k] = np.minimum(p[tuple(lo)], p[tuple(hi)])
    return out


def interior_mask(F, phi, sources):
    """Finite, reachable, non-source nodes with F > 0."""
    m = np.isfinite(phi) & (np.asarray(F) > 0)
    m.flat[np.asarray(sources, dtype=np.int64)] = False
    return m


def equation_residual(F, h, phi, sources) -> float:
    """max over interior nodes of |sum_k ((phi-a_k)^+)^2 - H^2|, relative to the
    size of its rounding error (see below)."""
    F = np.asarray(F, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    a = axis_minima(phi)
    m = interior_mask(F, phi, sources)
    if not m.any():
        return 0.0
    H = h / F[m]
    d = np.maximum(phi[m][None, :] - a[:, m], 0.0)
    d = np.where(np.isfinite(d), d, 0.0)
    r = (d * d).sum(axis=0) - H * H
    # rounding of phi and a_k perturbs each difference by ~eps*|phi|, so the
    # residual is measured against 2|phi| sum_k d_k + H^2
    scale = 2.0 * np.abs(phi[m]) * d.sum(axis=0) + H * H
    return float(np.max(np.abs(r) / scale))


def causality_ok(F, phi, sources) -> bool:
    """Every finite non-source node has a neighbour with strictly smaller phi."""
    phi = np.asarray(phi, dtype=np.float64)
    a = axis_minima(phi).min(axis=0)
    m = interior_mask(F, phi, sources)
    return bool(np.all(a[m] < phi[m]))


def local_bounds_ok(F, h, phi, sources, rtol: float = 1e-12) -> bool:
    """a_1 + H/sqrt(d) <= phi <= a_1 + H at every interior node."""
    F = np.asarray(F, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    a1 = axis_minima(phi).min(axis=0)
    m = interior_mask(F, phi, sources)
    H = h / F[m]
    lo = a1[m] + H / np.sqrt(phi.ndim)
    hi = a1[m] + H
    tol = rtol * np.maximum(np.abs(phi[m]), 1.0)
    return bool(np.all(phi[m] >= lo - tol) and np.all(phi[m] <= hi + tol))


def unreachable_mask(F, sources) -> np.ndarray:
    """Nodes not connected to any source through cells with F > 0 (flood fill);
    sources themselves are always reached."""
    F = np.asarray(F)
    reach = np.zeros(F.shape, dtype=bool)
    src = np.asarray(sources, dtype=np.int64)
    reach.flat[src] = True
    frontier = reach.copy()
    passable = F > 0
    while frontier.any():
        grow = np.zeros_like(reach)
        for k in range(F.ndim):
            for sh in (1, -1):
                r = np.roll(frontier, sh, axis=k)
                idx = [slice(None)] * F.ndim
                idx[k] = 0 if sh == 1 else -1
                r[tuple(idx)] = False
                grow |= r
        grow &= passable & ~reach
        reach |= grow
        frontier = grow
    return ~reach


def upwind_signature(phi: np.ndarray) -> np.ndarray:
    """Per node and axis: flat index of the upwind neighbour used by the
    Godunov update (a_k < phi_i), else -1.  Ties pick the lower index."""
    phi = np.asarray(phi, dtype=np.float64)
    n = phi.size
    idx = np.arange(n).reshape(phi.shape)
    sig = np.full((phi.ndim,) + phi.shape, -1, dtype=np.int64)
    for k in range(phi.ndim):
        pad = [(0, 0)] * phi.ndim
        pad[k] = (1, 1)
        p = np.pad(phi, pad, constant_values=np.inf)
        q = np.pad(idx, pad, constant_values=-1)
        lo = [slice(None)] * phi.ndim
        hi = [slice(None)] * phi.ndim
        lo[k] = slice(0, -2)
        hi[k] = slice(2, None)
        plo, phi_hi = p[tuple(lo)], p[tuple(hi)]
        qlo, qhi = q[tuple(lo)], q[tuple(hi)]
        use_lo = plo <= phi_hi
        amin = np.where(use_lo, plo, phi_hi)
        jmin = np.where(use_lo, qlo, qhi)
        sig[k] = np.where(amin < phi, jmin, -1)
    return sig
