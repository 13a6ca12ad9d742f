"""The differentiation workload at full size: 192^3 float32, layered speed
F(z) = 1.5 + 0.02 z with ten Gaussian anomalies, source at the top centre,
64 receivers on the bottom face, travel-time misfit loss

    L(F) = sum_r (phi_r(F) - t_obs,r)^2,   t_obs = phi(F_obs),

with F_obs the same field with the anomaly signs flipped.  phi and t_obs are
solved on the GPU (eik_solve) and checked against the float64 oracle; dL/dF
comes from torch autograd through EikonalFn (eik_adjoint).  Checks of dL/dF:

  * node by node against the oracle's reverse sweep on the GPU's own phi and
    the same dL/dphi, within the derived float32 rounding bound
    (tests/oracle_checks.py);
  * against central finite differences of the float64 oracle solve
    (dF = 1e-4 F_c) on 20 seeded cells, relative error <= 1e-3 for the float32
    GPU gradient and <= 1e-6 for the float64 oracle adjoint.  The cells are
    drawn from the cells whose gradient a float64 difference quotient can
    resolve (above its rounding floor, see below): the gradient is exactly
    zero off the receivers' upwind cones (most of the grid) and decays to
    1e-24 and below at their edges, where drawn cells would test nothing (the
    node-by-node check covers them).  A cell is
    excluded, and counted, when some node with a nonzero adjoint state uses a
    different upwind stencil in the F + dF and F - dF solves (L is not
    differentiable there);
  * the Euler identity sum_i F_i dL/dF_i = -sum_r 2 (phi_r - t_obs,r) phi_r
    (phi(cF) = phi(F)/c with zero-valued sources).
"""

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import workloads as W
from tests import helpers as H
from tests.oracle_checks import check_fp32_adjoint, fixed_point_ulps

torch = pytest.importorskip("torch")
eik = pytest.importorskip("paper_2106_15869_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _gate_phi(got, ref, F, h, src, what):
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(got)), what
    err = np.max(np.abs(got[fin].astype(np.float64) - ref[fin])) / ref[fin].max()
    ulps = fixed_point_ulps(F, h, got, src)
    print(f"[{what}] max err {err:.3e} of max phi, fixed point {ulps.max():.2f} ulp", flush=True)
    assert err <= 1e-5
    assert ulps.max() <= 4.0


def test_layered_192_misfit_gradient():
    n = 192
    P = W.layered_3d(n)
    F_obs = P.meta["F_obs"]
    rec = P.receivers
    src = P.sources
    print(f"[case] layered {n}^3 misfit, {len(rec)} receivers", flush=True)

    # observed travel times phi(F_obs), on the GPU, checked against the oracle
    t_obs = eik.solve(torch.from_numpy(F_obs).to(DEV), P.h, src)
    t_np = t_obs.cpu().numpy()
    t64 = oracle.fmm(F_obs.astype(np.float64), P.h, src)
    _gate_phi(t_np, t64, F_obs, P.h, src, "t_obs")

    # forward + misfit loss + backward through autograd
    F = torch.from_numpy(P.F).to(DEV).requires_grad_(True)
    phi = eik.EikonalFn.apply(F, P.h, src)
    rec_t = torch.from_numpy(rec).to(DEV)
    L = ((phi.reshape(-1)[rec_t] - t_obs.reshape(-1)[rec_t]) ** 2).sum()
    L.backward()
    grad = F.grad.cpu().numpy().astype(np.float64)
    phi_np = phi.detach().cpu().numpy()
    phi64 = oracle.fmm(P.F.astype(np.float64), P.h, src)
    _gate_phi(phi_np, phi64, P.F, P.h, src, "phi")

    # dL/dphi as autograd formed it (float32: 2 (phi_r - t_r)), for the oracle
    g32 = np.zeros(P.F.size, dtype=np.float32)
    g32[rec] = np.float32(2) * (phi_np.ravel()[rec] - t_np.ravel()[rec])
    g = g32.reshape(P.F.shape).astype(np.float64)
    F64 = P.F.astype(np.float64)
    check_fp32_adjoint(grad, F64, P.h, src, phi_np, g, label=" misfit 192^3")

    # Euler identity on the GPU gradient
    rhs = -float(np.sum(g.ravel()[rec] * phi_np.ravel()[rec].astype(np.float64)))
    scale = float(np.sum(np.abs(g.ravel()[rec] * phi_np.ravel()[rec])))
    lhs = float(np.sum(F64 * grad))
    print(f"[euler] sum F dL/dF = {lhs:.6e}, -sum g phi = {rhs:.6e}", flush=True)
    assert abs(lhs - rhs) <= 1e-4 * scale

    # central finite differences of the float64 oracle
    t64r = t64.ravel()[rec]

    def loss64(Fx):
        p = oracle.fmm(Fx, P.h, src)
        return float(np.sum((p.ravel()[rec] - t64r) ** 2)), p

    g64 = np.zeros(P.F.size)
    g64[rec] = 2.0 * (phi64.ravel()[rec] - t64r)
    g64 = g64.reshape(P.F.shape)
    d64, lam64 = oracle.adjoint(F64, P.h, src, phi64, g64, return_lambda=True)
    # A float64 central difference resolves a gradient only above its rounding
    # floor: the solve rounds each receiver time at ~eps64 phi_r, so L_+ - L_-
    # carries up to ~2 eps64 S (S = sum_r |g_r| phi_r) and the quotient
    # eps64 S / dF with dF = 1e-4 F_c.  Cells are drawn where that is at most
    # 1e-5 of the gradient, |F_c dL/dF_c| >= 2.3e-7 S, here >= 1e-6 S.
    S = float(np.sum(np.abs(g64.ravel()[rec]) * phi64.ravel()[rec]))
    support = np.flatnonzero((d64.ravel() != 0.0) & (np.abs(d64.ravel() * F64.ravel()) >= 1e-6 * S))
    support = np.setdiff1d(support, src)
    influence = np.flatnonzero(lam64.ravel() != 0.0)
    r = np.random.default_rng(W.BASE_SEED + 4)
    cells = np.sort(r.choice(support, size=20, replace=False))
    print(f"[fd] {int(np.count_nonzero(d64))} cells with a nonzero gradient, {support.size} above the "
          f"difference quotient's rounding floor; checking {cells.size}", flush=True)

    def sig(p):
        return H.upwind_signature(p).reshape(p.ndim, -1)[:, influence]

    def fd(c):
        dF = 1e-4 * F64.flat[c]
        Fp = F64.copy()
        Fp.flat[c] += dF
        Lp, pp = loss64(Fp)
        Fp.flat[c] = F64.flat[c] - dF
        Lm, pm = loss64(Fp)
        switched = not np.array_equal(sig(pp), sig(pm))
        return (Lp - Lm) / (2 * dF), switched

    workers = max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        res = list(ex.map(fd, cells))
    checked = excluded = 0
    worst32 = worst64 = 0.0
    for c, (v, switched) in zip(cells, res):
        if switched:
            excluded += 1
            continue
        e32 = abs(grad.flat[c] - v) / abs(v)
        e64 = abs(d64.flat[c] - v) / abs(v)
        worst32, worst64 = max(worst32, e32), max(worst64, e64)
        assert e32 <= 1e-3, (int(c), grad.flat[c], v)
        assert e64 <= 1e-6, (int(c), d64.flat[c], v)
        checked += 1
    print(f"[fd] checked {checked}, excluded (stencil switch) {excluded}; worst relative error "
          f"float32 GPU {worst32:.3e}, float64 oracle {worst64:.3e}", flush=True)
    assert checked >= 15
