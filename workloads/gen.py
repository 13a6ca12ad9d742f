"""Seeded synthetic workloads.

Every generator is deterministic in its seed (numpy PCG64).  Fields are built in
float64 and cast to the requested storage dtype at the end, so the oracle can
consume the *same* rounded values upcast to float64.

Workload recipes (shapes, value distributions) stand in for the paper's
experiments, which use 2D analytic speed fields and a barrier map on grids of
200^2 to 4000^2 (Results section, Examples 1-5); see the module docstrings of
each generator for the exact recipe.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

BASE_SEED = 2106


@dataclass
class Problem:
    """One eikonal problem instance: ||grad phi|| = 1/F on a uniform grid."""

    name: str
    F: np.ndarray                 # speed, C-order, last axis fastest
    h: float                      # isotropic grid spacing
    sources: np.ndarray           # int64 flat C-order indices
    source_values: Optional[np.ndarray] = None  # float64, None -> all zero
    eps: float = 0.0
    receivers: Optional[np.ndarray] = None      # int64 flat indices (adjoint losses)
    meta: dict = field(default_factory=dict)

    @property
    def dims(self) -> Tuple[int, ...]:
        return tuple(int(d) for d in self.F.shape)

    @property
    def n(self) -> int:
        return int(self.F.size)


def flat_index(dims: Sequence[int], coord: Sequence[int]) -> int:
    idx = 0
    for d, c in zip(dims, coord):
        idx = idx * int(d) + int(c)
    return idx


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _gaussian_filter_periodic(g: np.ndarray, sigma: float) -> np.ndarray:
    """Periodic Gaussian filter (std `sigma` cells) applied in Fourier space."""
    k2 = np.zeros(g.shape, dtype=np.float64)
    for ax, n in enumerate(g.shape):
        shape = [1] * g.ndim
        shape[ax] = n
        k = np.fft.fftfreq(n).reshape(shape)
        k2 = k2 + k * k
    kernel = np.exp(-2.0 * np.pi ** 2 * sigma ** 2 * k2)
    return np.real(np.fft.ifftn(np.fft.fftn(g) * kernel))


def lognormal_field(shape: Sequence[int], seed: int, sigma: float = 8.0,
                    dtype=np.float32) -> np.ndarray:
    """F = exp(0.5 g), g = i.i.d. N(0,1) noise, periodic Gaussian filter of std
    `sigma` cells, renormalised to zero mean and unit variance."""
    g = _rng(seed).standard_normal(tuple(shape))
    g = _gaussian_filter_periodic(g, sigma)
    g = (g - g.mean()) / g.std()
    return np.exp(0.5 * g).astype(dtype)


def maze_field(shape: Sequence[int], seed: int, block: int = 8, p: float = 0.3,
               slow: float = 0.001, free_coord: Optional[Sequence[int]] = None,
               dtype=np.float32) -> np.ndarray:
    """Blocks of `block`^d cells; each block is an obstacle (F = `slow`) with
    probability `p`, else free (F = 1).  The block holding `free_coord` is forced
    free."""
    nb = [-(-int(n) // block) for n in shape]
    obst = _rng(seed).random(tuple(nb)) < p
    if free_coord is not None:
        obst[tuple(int(c) // block for c in free_coord)] = False
    Fb = np.where(obst, slow, 1.0)
    F = Fb
    for ax in range(len(shape)):
        F = np.repeat(F, block, axis=ax)
    F = F[tuple(slice(0, int(n)) for n in shape)]
    return np.ascontiguousarray(F).astype(dtype)


def layered_anomaly_field(shape: Sequence[int], seed: int, n_anom: int = 10,
                          amp: float = 0.3, sigma_range=(6.0, 15.0),
                          flip_signs: bool = False, dtype=np.float32) -> np.ndarray:
    """F(z) = 1.5 + 0.02 z (z = axis 0) plus `n_anom` Gaussian anomalies of
    amplitude +-`amp`, std uniform in `sigma_range` cells, seeded centres.
    `flip_signs` negates every anomaly (the 'observed' field of a travel-time
    misfit)."""
    r = _rng(seed)
    nd = len(shape)
    centres = np.stack([r.uniform(0, n - 1, n_anom) for n in shape], axis=1)
    sigmas = r.uniform(sigma_range[0], sigma_range[1], n_anom)
    signs = np.where(r.random(n_anom) < 0.5, -1.0, 1.0)
    if flip_signs:
        signs = -signs
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    F = 1.5 + 0.02 * grids[0]
    for m in range(n_anom):
        d2 = sum((grids[a] - centres[m, a]) ** 2 for a in range(nd))
        F = F + signs[m] * amp * np.exp(-d2 / (2.0 * sigmas[m] ** 2))
    return F.astype(dtype)


def receivers_on_face(shape: Sequence[int], count: int, seed: int, axis: int = 0,
                      side: int = -1) -> np.ndarray:
    """`count` distinct seeded receiver nodes on the face axis=`side`."""
    r = _rng(seed)
    shape = [int(s) for s in shape]
    face_shape = [n for a, n in enumerate(shape) if a != axis]
    m = int(np.prod(face_shape))
    pick = r.choice(m, size=min(count, m), replace=False)
    pick.sort()
    coords = np.unravel_index(pick, face_shape)
    fixed = shape[axis] - 1 if side == -1 else 0
    out = []
    for k in range(len(pick)):
        c = []
        j = 0
        for a in range(len(shape)):
            if a == axis:
                c.append(fixed)
            else:
                c.append(int(coords[j][k]))
                j += 1
        out.append(flat_index(shape, c))
    return np.asarray(out, dtype=np.int64)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def tiny_constant(dtype=np.float64) -> Problem:
    """2D 64x64, h = 1, F = 1, one point source at (32, 32), eps = 1e-12."""
    dims = (64, 64)
    F = np.ones(dims, dtype=dtype)
    src = np.array([flat_index(dims, (32, 32))], dtype=np.int64)
    return Problem("tiny_constant_64x64", F, 1.0, src, eps=1e-12)


def lognormal_2d(n: int = 4096, seed: int = BASE_SEED, dtype=np.float32,
                 sigma: float = 8.0) -> Problem:
    """2D n x n, h = 1/n, lognormal speed F = exp(0.5 g) (filtered noise,
    sigma = 8 cells), single source at (0, 0)."""
    F = lognormal_field((n, n), seed, sigma=sigma, dtype=dtype)
    src = np.array([0], dtype=np.int64)
    return Problem(f"lognormal_2d_{n}x{n}", F, 1.0 / n, src, eps=0.0)


def maze_3d(n: int = 256, seed: int = BASE_SEED, dtype=np.float32, block: int = 8,
            p: float = 0.3) -> Problem:
    """3D n^3, h = 1, maze of block^3 obstacles (F = 0.001, probability p) in a
    free medium (F = 1); source (0,0,0), its block forced free."""
    dims = (n, n, n)
    F = maze_field(dims, seed, block=block, p=p, free_coord=(0, 0, 0), dtype=dtype)
    src = np.array([0], dtype=np.int64)
    return Problem(f"maze_3d_{n}^3", F, 1.0, src, eps=0.0)


def layered_3d(n: int = 192, seed: int = BASE_SEED, dtype=np.float32,
               n_receivers: int = 64) -> Problem:
    """3D n^3, h = 1, F(z) = 1.5 + 0.02 z plus 10 Gaussian anomalies; source at
    the top-centre (0, n/2, n/2); receivers on the bottom face z = n-1."""
    dims = (n, n, n)
    F = layered_anomaly_field(dims, seed, dtype=dtype)
    src = np.array([flat_index(dims, (0, n // 2, n // 2))], dtype=np.int64)
    rec = receivers_on_face(dims, n_receivers, seed + 1, axis=0, side=-1)
    P = Problem(f"layered_3d_{n}^3", F, 1.0, src, eps=0.0, receivers=rec)
    P.meta["F_obs"] = layered_anomaly_field(dims, seed, flip_signs=True, dtype=dtype)
    return P


def batch_2d(count: int = 256, seed: int = BASE_SEED, lo: int = 128, hi: int = 2048,
             dtype=np.float32, n_receivers: int = 16) -> List[Problem]:
    """`count` independent 2D lognormal problems with side lengths uniform in
    [lo, hi], 1-8 distinct random point sources each, h = 1/max(ny, nx),
    receivers on the last row.  Instance i uses seed + i."""
    out = []
    for i in range(count):
        r = _rng(seed + i)
        ny, nx = (int(v) for v in r.integers(lo, hi + 1, size=2))
        k = int(r.integers(1, 9))
        src = np.sort(r.choice(ny * nx, size=k, replace=False)).astype(np.int64)
        F = lognormal_field((ny, nx), seed + i, dtype=dtype)
        rec = receivers_on_face((ny, nx), n_receivers, seed + 10_000 + i, axis=0, side=-1)
        out.append(Problem(f"batch_{i}_{ny}x{nx}", F, 1.0 / max(ny, nx), src,
                           eps=0.0, receivers=rec))
    return out


def random_problem(seed: int, ndim: int, max_side: int, dtype=np.float64,
                   f_lo: float = 1e-3, f_hi: float = 1e3, max_sources: int = 8,
                   zero_frac: float = 0.0, h: Optional[float] = None) -> Problem:
    """Small fuzz case: random shape, log-uniform F in [f_lo, f_hi] (a fraction
    `zero_frac` of cells set to the barrier value 0), 1..max_sources sources."""
    r = _rng(seed)
    dims = tuple(int(v) for v in r.integers(1, max_side + 1, size=ndim))
    n = int(np.prod(dims))
    F = np.exp(r.uniform(np.log(f_lo), np.log(f_hi), size=dims))
    if zero_frac > 0:
        F[r.random(dims) < zero_frac] = 0.0
    k = int(r.integers(1, min(max_sources, n) + 1))
    src = np.sort(r.choice(n, size=k, replace=False)).astype(np.int64)
    hh = float(h) if h is not None else float(r.uniform(0.1, 2.0))
    return Problem(f"random_{ndim}d_{seed}", F.astype(dtype), hh, src, eps=0.0)


# ---------------------------------------------------------------------------
# The paper's own examples (Results section), on n x n nodes over [-10, 10]^2
# ---------------------------------------------------------------------------
PAPER_SIZES = (200, 500, 1000, 2000, 4000)


def _paper_grid(n: int):
    """Node coordinates x_j = -10 + j h, h = 20 / (n - 1); axis 0 is y, axis 1 x."""
    h = 20.0 / (n - 1)
    c = -10.0 + h * np.arange(n)
    return h, c[:, None], c[None, :]


def _circle_band(F, h, ys, xs, circles):
    """Nodes within one spacing of a circle become fixed sources valued
    |dist - R| / F (first-order arrival time from the circle); a node near
    several circles keeps the smallest value."""
    best = np.full(F.shape, np.inf)
    for (cx, cy, R) in circles:
        d = np.abs(np.sqrt((xs - cx) ** 2 + (ys - cy) ** 2) - R)
        best = np.where(d <= h, np.minimum(best, d), best)
    idx = np.flatnonzero(np.isfinite(best))
    Fv = F.ravel()[idx].astype(np.float64)
    with np.errstate(divide="ignore"):
        vals = np.where(Fv > 0, best.ravel()[idx] / np.where(Fv > 0, Fv, 1.0), 0.0)
    return idx.astype(np.int64), vals


def paper_example(k: int, n: int, dtype=np.float32) -> Problem:
    """Examples 1, 2, 3 and 5 of the paper on an n x n grid over [-10, 10]^2.

    1: F = 1, circle R = 3 at the origin.
    2: F = 1, circles R = 3 at (2, -5) and R = 1.5 at (-2, 5).
    3: F = 1 on [3, 7]^2 and 0.01 elsewhere (Eq 7), circles R = 0.5 at (-5, 5)
       and (5, -5).
    5: F = sin^2 x + sin^2 y + 0.3 (Eq 9), circle R = 0.5 at the origin.
    The circles enter as fixed sources on the nodes within one spacing of
    them (the paper does not state its discretisation of the circles)."""
    h, ys, xs = _paper_grid(n)
    if k == 1:
        F = np.ones((n, n))
        circles = [(0.0, 0.0, 3.0)]
    elif k == 2:
        F = np.ones((n, n))
        circles = [(2.0, -5.0, 3.0), (-2.0, 5.0, 1.5)]
    elif k == 3:
        inside = (xs >= 3) & (xs <= 7) & (ys >= 3) & (ys <= 7)
        F = np.where(inside, 1.0, 0.01) * np.ones((n, n))
        circles = [(-5.0, 5.0, 0.5), (5.0, -5.0, 0.5)]
    elif k == 5:
        F = np.sin(xs) ** 2 + np.sin(ys) ** 2 + 0.3
        circles = [(0.0, 0.0, 0.5)]
    else:
        raise ValueError("examples 1, 2, 3 and 5 are available (example 4's map is not)")
    F = F.astype(dtype)
    src, vals = _circle_band(F, h, ys, xs, circles)
    return Problem(f"paper_ex{k}_{n}", F, h, src, source_values=vals,
                   meta={"example": k, "circles": circles})
