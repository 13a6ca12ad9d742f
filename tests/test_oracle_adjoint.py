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


def test_adjoint_state_1d_closed_form():
    """On a strip every node depends on its predecessor alone with weight 1,
    so the adjoint state is lambda_j = g_j + sum of g over the nodes further
    from the source (and the source collects everything on its sides)."""
    r = np.random.default_rng(8)
    n = 30
    F = np.exp(r.uniform(-1, 1, size=(1, n)))
    s = 11
    phi = oracle.fmm(F, 0.5, [s])
    g = np.zeros_like(F)
    g[0, r.choice(n, size=9, replace=False)] = r.uniform(-2, 2, size=9)
    _, lam = oracle.adjoint(F, 0.5, [s], phi, g, return_lambda=True)
    want = np.empty(n)
    for j in range(n):
        want[j] = g[0, j:].sum() if j > s else g[0, :j + 1].sum() if j < s else g[0].sum()
    np.testing.assert_allclose(lam[0], want, rtol=0, atol=1e-13)


def test_adjoint_state_linearity_and_gradient():
    """dL/dF = D lambda with lambda linear in dL/dphi: the adjoint of g1 + 2 g2
    is the sum of the two, and dL/dF / lambda is the same per node for both."""
    P = W.lognormal_2d(24, dtype=np.float64)
    phi = oracle.fmm(P.F, P.h, P.sources)
    r = np.random.default_rng(4)
    g1, g2 = r.normal(size=phi.shape), r.normal(size=phi.shape)
    d1, l1 = oracle.adjoint(P.F, P.h, P.sources, phi, g1, return_lambda=True)
    d2, l2 = oracle.adjoint(P.F, P.h, P.sources, phi, g2, return_lambda=True)
    d3, l3 = oracle.adjoint(P.F, P.h, P.sources, phi, g1 + 2 * g2, return_lambda=True)
    np.testing.assert_allclose(l3, l1 + 2 * l2, rtol=1e-12, atol=1e-12 * np.abs(l3).max())
    np.testing.assert_allclose(d3, d1 + 2 * d2, rtol=1e-12, atol=1e-12 * np.abs(d3).max())
    m = np.abs(l1) > 1e-6
    m.flat[P.sources] = False
    np.testing.assert_allclose(d1[m] / l1[m], d2[m] / l2[m], rtol=1e-9)


def test_adjoint_threads_match_serial():
    """The oracle's adjoint is called from thread pools (the batch baseline):
    concurrent calls on grids of different sizes give the serial results."""
    from concurrent.futures import ThreadPoolExecutor
    rng = np.random.default_rng(11)
    probs = []
    for _ in range(16):
        n, m = int(rng.integers(16, 120)), int(rng.integers(16, 120))
        F = np.exp(0.3 * rng.normal(size=(n, m)))
        probs.append((F, np.array([int(rng.integers(0, n * m))])))

    def one(P):
        F, src = P
        p = oracle.fmm(F, 1.0, src)
        return oracle.adjoint(F, 1.0, src, p, np.ones(F.shape))
    serial = [one(P) for P in probs]
    for _ in range(3):
        with ThreadPoolExecutor(max_workers=8) as ex:
            par = list(ex.map(one, probs))
        assert all(np.array_equal(a, b) for a, b in zip(serial, par))
