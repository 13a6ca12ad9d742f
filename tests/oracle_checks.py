"""Checks of GPU outputs that use the float64 oracle on the GPU's own result.

fixed_point_ulps: how far a float32 solution is from being a fixed point of
the exact local solve (Eq 4 / Eq 6), node by node, in float32 ulps.

fp32_adjoint_bound / check_fp32_adjoint: rounding bound of a float32 adjoint,
node by node.

chain_bound: bound on the distance of a float32 solution from the float64
fixed point, from the float32 solution's own per-node residual.

The GPU adjoint and the float64 oracle adjoint are compared on the SAME
solution phi (the GPU's float32 output, upcast exactly).  Both then use the
same upwind stencil at every node (the stencil is read off phi, the lower
index winning a tie on both sides), so they solve the same linear system

    lambda = g + M^T lambda,   dL/dF = D lambda,
    M_{i,j_k} = c_ik = w_ik / W_i,  W_i = sum_k w_ik,  w_ik = phi_i - phi_{j_k},
    D_i = -(h/F_i)^2 / (F_i W_i)

(the derivative of the Eq 4 / Eq 6 fixed point), and differ only by the
float32 rounding of the GPU's arithmetic.  With u = 2^-24:

* a coefficient c_ik carries at most (3 + ND) u: w_ik one rounding (two more
  with per-axis spacing), W_i ND - 1, the division one;
* the GPU recomputes lambda_j = g_j + sum_i c_ij lambda_i from the final
  lambda_i (a node is recomputed whenever one of its inputs changes), one
  rounding per product and up to 2 ND additions;
* so, with e_j the error of lambda_j and kappa = (7 + 2 ND) u,
      e_j <= sum_i c_ij e_i + kappa (|g_j| + sum_i c_ij |lambda_i|),
  and by induction over the causal order e_j <= kappa nu_j, where
      labs = |g| + M^T labs   (the adjoint of |g|) and
      nu   = labs + M^T nu    (the adjoint of labs);
  nu_j sums every contribution to lambda_j weighted by its path length + 1;
* dL/dF_j = D_j lambda_j adds at most 12 u |D_j| labs_j (D_j's own roundings
  and the product).

Hence |dL/dF_gpu - dL/dF_oracle| <= u |D| ((7 + 2 ND) nu + 12 labs) per node,
computed here with two more oracle adjoint solves (to first order in u; the
oracle's own float64 rounding is 2^29 times smaller).

The relative model holds only inside float32's normal range.  Below 2^-126 a
rounded result carries an absolute error of up to 2^-126 (flushed to zero) or
half a subnormal step (gradual underflow), whatever its size; gradients of
cells far upwind of every receiver fall there (2D lognormal batch grids reach
1e-46).  So every rounding also adds at most tau = 2^-126 absolute: at most
2 ND + 2 of them per lambda_j, carried like the relative terms, i.e.
(2 ND + 2) tau nu1_j with nu1 = 1 + M^T nu1 (the adjoint of the all-ones
loss gradient), and one more for the final product, which gives

    |dL/dF_gpu - dL/dF_oracle| <= u |D| ((7 + 2 ND) nu + 12 labs)
                                  + tau (1 + (2 ND + 2) |D| nu1).

The floor is below 1e-30 for every grid here, far under any normal-range
value's relative term.
"""

from __future__ import annotations

import numpy as np

import oracle

U32 = 2.0 ** -24
TINY32 = 2.0 ** -126   # smallest normal float32: the absolute floor of one rounding


def fixed_point_ulps(F, h, phi, sources) -> np.ndarray:
    """|phi_i - G_i(phi)| / ulp_f32(phi_i) over finite non-source nodes with
    F > 0, G evaluated in float64 by the oracle on the float32 values.

    A float32 run of Algorithm 2 with eps = 0 ends where no node's float32
    update lies below its value and every value is a float32 update of
    neighbour values at least as large; the float32 root is monotone in its
    inputs only up to its own rounding, so the distance is a few ulps, not
    zero (the oracle's float32 emulation of Algorithm 2 ends at up to 2.94 ulp
    on a 48^3 maze, where H = 1000 in the obstacles, and 0.8 ulp on smooth
    fields)."""
    F64 = np.asarray(F, dtype=np.float64)
    p = np.asarray(phi)
    G = oracle.apply_local(F64, h, p.astype(np.float64))
    m = np.isfinite(p) & (F64 > 0)
    m.flat[np.asarray(sources, dtype=np.int64)] = False
    ulp = np.spacing(np.abs(p[m]).astype(np.float32)).astype(np.float64)
    return np.abs(p[m].astype(np.float64) - G[m]) / ulp


def fp32_adjoint_bound(F, h, sources, phi, g, spacing=None) -> np.ndarray:
    """Per-node bound on |float32 GPU adjoint - float64 oracle adjoint|, both on
    the solution `phi`, for the loss gradient `g` (see the module docstring)."""
    nd = np.ndim(F)
    F64 = np.asarray(F, dtype=np.float64)
    p = np.asarray(phi, dtype=np.float64)
    ga = np.abs(np.asarray(g, dtype=np.float64))
    d_abs, labs = oracle.adjoint(F64, h, sources, p, ga, spacing=spacing, return_lambda=True)
    d_nu = oracle.adjoint(F64, h, sources, p, labs, spacing=spacing)
    d_one = oracle.adjoint(F64, h, sources, p, np.ones_like(p), spacing=spacing)
    return (U32 * ((7 + 2 * nd) * np.abs(d_nu) + 12.0 * np.abs(d_abs))
            + TINY32 * (1.0 + (2 * nd + 2) * np.abs(d_one)))


def check_fp32_adjoint(got, F, h, sources, phi, g, spacing=None, label=""):
    """Assert the float32 adjoint `got` matches the oracle adjoint on the same
    phi within the per-node bound; returns (max relative error, max error /
    bound) for the record."""
    want = oracle.adjoint(np.asarray(F, dtype=np.float64), h, sources, np.asarray(phi, dtype=np.float64),
                          np.asarray(g, dtype=np.float64), spacing=spacing)
    bound = fp32_adjoint_bound(F, h, sources, phi, g, spacing=spacing)
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - want)
    bad = err > bound + 1e-300
    scale = max(float(np.abs(want).max()), 1e-300)
    ratio = float(np.max(err / np.maximum(bound, 1e-300)))
    print(f"[adjoint{label}] max|err| {err.max():.3e} = {err.max() / scale:.3e} of max|dL/dF|; "
          f"max err/bound {ratio:.3e}; nodes over the bound {int(bad.sum())}", flush=True)
    assert not bad.any(), (int(bad.sum()), float(err[bad].max()), float(bound[bad].min()))
    return err.max() / scale, ratio


def chain_bound(F, h, sources, phi, source_values=None) -> float:
    """Bound on max |phi - phi64| (phi64 the float64 fixed point) from the
    residual of `phi` (float32) under the exact local solve.

    The Godunov update G (Eq 4 / Eq 6) is monotone, G(x + c) = G(x) + c for a
    constant c added to every input, and G_i depends only on neighbours whose
    value is below G_i (an input at or above the root does not enter it).  So
    at node i, with e = phi - phi64 and r_i = |phi_i - G_i(phi)|:
        e_i <= max(e_k over neighbours k below phi64_i) + r_i,   and
       -e_i <= max(-e_k over neighbours k below phi_i)  + r_i;
    a chain of such neighbours ends at a source, and each step drops by at
    least H_k / sqrt(d) >= h / (F_max sqrt(d)) (the local lower bound
    a_1 + H / sqrt(d) <= G).  Hence
        max |e| <= (sqrt(d) F_max max(phi) / h) max r + max |source rounding|.
    """
    F64 = np.asarray(F, dtype=np.float64)
    p = np.asarray(phi)
    G = oracle.apply_local(F64, h, p.astype(np.float64))
    m = np.isfinite(p) & (F64 > 0)
    m.flat[np.asarray(sources, dtype=np.int64)] = False
    r = float(np.max(np.abs(p[m].astype(np.float64) - G[m]))) if m.any() else 0.0
    top = float(np.max(p[np.isfinite(p)].astype(np.float64)))
    steps = np.sqrt(np.ndim(F64)) * float(F64.max()) * top / h
    vals = np.zeros(len(np.ravel(sources))) if source_values is None else np.asarray(source_values, dtype=np.float64)
    src = float(np.max(np.abs(vals.astype(np.float32).astype(np.float64) - vals))) if vals.size else 0.0
    return steps * r + src
