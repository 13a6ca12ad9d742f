"""Pins of the oracle adjoint (dL/dF of the converged discrete system)."""

import numpy as np
import pytest

import oracle
import workloads as W
from tests import helpers as H


def test_adjoint_1d_closed_form():
    """On a strip, phi_n = sum_{j on path} h/F_j, so dphi_n/dF_j = -h/F_j^2
    for path cells j (excluding the source) and 0 elsewhere."""
    r = np.random.default_rng(3)
    n = 25
    F = np.exp(r.uniform(-1, 1, size=(1, n)))
    h = 0.37
    s = 6
    phi = oracle.fmm(F, h, [s])
    for tgt in (0, 5, 7, 24):
        g = np.zeros_like(F)
        g[0, tgt] = 1.0
        d = oracle.adjoint(F, h, [s], phi, g)
        want = np.zeros(n)
        lo, hi = (s + 1, tgt + 1) if tgt > s else (tgt, s)
        want[lo:hi] = -h / F[0, lo:hi] ** 2
        np.testing.assert_allclose(d[0], want, rtol=1e-14, atol=0)


@pytest.mark.parametrize("P", [W.lognormal_2d(40, dtype=np.float64),
                               W.random_problem(5, 3, 9),
                               W.layered_3d(12, dtype=np.float64, n_receivers=8)],
                         ids=lambda P: P.name)
def test_adjoint_euler_identity(P):
    """phi(cF) = phi(F)/c for zero-valued sources, hence sum_i F_i dphi_x/dF_i
    = -phi_x, and for L = sum_r c_r phi_r: sum_i F_i dL/dF_i = -L."""
    phi = oracle.fmm(P.F, P.h, P.sources)
    r = np.random.default_rng(0)
    g = np.zeros_like(phi)
    fin = np.flatnonzero(np.isfinite(phi.ravel()))
    pick = r.choice(fin, size=min(10, fin.size), replace=False)
    g.flat[pick] = r.uniform(0.5, 2.0, size=pick.size)
    d = oracle.adjoint(P.F, P.h, P.sources, phi, g)
    L = float((g * np.where(np.isfinite(phi), phi, 0)).sum())
    assert float((P.F * d).sum()) == pytest.approx(-L, rel=1e-11)


def _fd_check(P, ncells, seed, rel_delta=1e-6, tol=1e-5):
    phi = oracle.fmm(P.F, P.h, P.sources)
    r = np.random.default_rng(seed)
    fin = np.flatnonzero(np.isfinite(phi.ravel()))
    rec = r.choice(fin, size=min(12, fin.size), replace=False)
    wts = r.uniform(0.5, 2.0, size=rec.size)
    g = np.zeros_like(phi)
    g.flat[rec] = wts
    d = oracle.adjoint(P.F, P.h, P.sources, phi, g)

    def loss(F):
        p = oracle.fmm(F, P.h, P.sources)
        return float((p.flat[rec] * wts).sum()), p

    cand = np.setdiff1d(fin, P.sources)
    cells = r.choice(cand, size=min(ncells, cand.size), replace=False)
    checked = skipped = 0
    for c in cells:
        dF = rel_delta * P.F.flat[c]
        Fp = P.F.copy(); Fp.flat[c] += dF
        Fm = P.F.copy(); Fm.flat[c] -= dF
        Lp, pp = loss(Fp)
        Lm, pm = loss(Fm)
        # the loss is not differentiable where the upwind stencil switches
        if not np.array_equal(H.upwind_signature(pp), H.upwind_signature(pm)):
            skipped += 1
            continue
        fd = (Lp - Lm) / (2 * dF)
        scale = max(abs(fd), 1e-3 * np.abs(d).max(), 1e-300)
        assert abs(d.flat[c] - fd) <= tol * scale, (c, d.flat[c], fd)
        checked += 1
    assert checked >= ncells // 2, (checked, skipped)


def test_adjoint_matches_finite_differences_2d():
    _fd_check(W.lognormal_2d(32, dtype=np.float64), 30, 1)


def test_adjoint_matches_finite_differences_3d():
    _fd_check(W.layered_3d(10, dtype=np.float64, n_receivers=6), 30, 2)
