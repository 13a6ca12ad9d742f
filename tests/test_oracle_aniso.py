"""Pins of the anisotropic local solve and grid solvers (Eq 5 with dx != dy,
Algorithm 1.2, and its 3D analogue): closed forms, the two-sided formula
Algorithm 1.2 prints (valid where both axes are upwind), the printed branch
thresholds (not valid), the residual, bisection, the isotropic limit, exact
axis values, brute-force sweeping, scaling, FIM, and the adjoint against
finite differences and the Euler identity."""

import numpy as np
import pytest

import oracle
from tests import helpers as H

R = np.random.default_rng(1212)


def residual(a, Hk, phi):
    return sum(((phi - ak) / hk) ** 2 for ak, hk in zip(a, Hk) if ak < phi) - 1.0


def test_closed_forms():
    assert oracle.godunov_aniso([0.0, 0.0], [1.0, 2.0]) == pytest.approx(2 / np.sqrt(5), rel=1e-15)
    assert oracle.godunov_aniso([0.0, 0.0, 0.0], [1.0, 2.0, 2.0]) == pytest.approx(np.sqrt(2 / 3), rel=1e-15)
    assert oracle.godunov_aniso([0.0, np.inf], [0.7, 3.0]) == 0.7
    assert oracle.godunov_aniso([np.inf, 5.0], [0.7, 3.0]) == 8.0
    assert oracle.godunov_aniso([0.0, 10.0, 1.0], [1.0, 1.0, 1.0]) == pytest.approx(1.0)  # one upwind axis


def _printed_alg12(ax, ay, dx, dy, f):
    """Algorithm 1.2 as printed (thresholds sqrt(dx^2 + dy^2) / f)."""
    lim = np.sqrt((dx * dx + dy * dy) / (f * f))
    if ax - ay > lim:
        return ay + dy / f
    if ax - ay < -lim:
        return ax + dx / f
    return (ax * dy * dy + ay * dx * dx + dx * dy * np.sqrt((dx * dx + dy * dy) / (f * f) - (ax - ay) ** 2)) / (
        dx * dx + dy * dy)


def test_two_sided_formula_of_alg12_where_valid():
    """Where both axes are upwind, Algorithm 1.2's two-sided expression is the
    root (a = (a_y, a_x) in dims order, H = (dy/f, dx/f))."""
    checked = 0
    for _ in range(500):
        dx, dy, f = R.uniform(0.2, 3.0), R.uniform(0.2, 3.0), R.uniform(0.2, 3.0)
        ax, ay = R.uniform(0, 2), R.uniform(0, 2)
        got = oracle.godunov_aniso([ay, ax], [dy / f, dx / f])
        if got > max(ax, ay):
            assert got == pytest.approx(_printed_alg12(ax, ay, dx, dy, f), rel=1e-13)
            checked += 1
    assert checked > 100


def test_printed_alg12_thresholds_do_not_solve_eq5():
    """The printed switch leaves the two-sided branch active where one axis is
    no longer upwind: with dx = dy = f = 1 and (a_x, a_y) = (1.2, 0) it
    returns a value below a_x; the exact root is a_y + dy/f = 1."""
    printed = _printed_alg12(1.2, 0.0, 1.0, 1.0, 1.0)
    assert printed < 1.2
    assert abs(residual([0.0, 1.2], [1.0, 1.0], printed)) > 1e-3
    assert oracle.godunov_aniso([0.0, 1.2], [1.0, 1.0]) == 1.0


@pytest.mark.parametrize("m", [2, 3])
def test_residual_and_bisection(m):
    for _ in range(300):
        a = R.uniform(0, 3, size=m)
        Hk = R.uniform(0.1, 3, size=m)
        phi = oracle.godunov_aniso(a, Hk)
        assert abs(residual(a, Hk, phi)) <= 1e-13
        # bisection on the monotone residual
        lo, hi = a.min(), a.min() + Hk[np.argmin(a)]
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if residual(a, Hk, mid) < 0:
                lo = mid
            else:
                hi = mid
        assert phi == pytest.approx(hi, abs=1e-12)


def test_isotropic_limit():
    """Equal spacings give the isotropic root; the weighted form rounds
    differently (the 1/H^2 weights), so a few ulps apart."""
    for _ in range(300):
        m = int(R.integers(2, 4))
        a = R.uniform(0, 3, size=m)
        h = R.uniform(0.1, 3)
        assert oracle.godunov_aniso(a, [h] * m) == pytest.approx(oracle.godunov(a, h), rel=2e-15, abs=1e-300)


def test_float32_version_close():
    for _ in range(200):
        a = R.uniform(0, 50, size=3).astype(np.float32)
        Hk = R.uniform(0.1, 3, size=3).astype(np.float32)
        g64 = oracle.godunov_aniso(a.astype(np.float64), Hk.astype(np.float64))
        g32 = oracle.godunov_aniso(a, Hk, dtype=np.float32)
        assert abs(float(g32) - g64) <= 4e-7 * max(abs(g64), 1.0)


def test_axis_values_exact_2d():
    dims = (21, 31)
    sp = (0.5, 1.25)  # (dy, dx)
    F = np.ones(dims)
    src = [10 * 31 + 15]
    phi = oracle.fmm(F, 1.0, src, spacing=sp)
    assert np.array_equal(phi[10, :], np.abs(np.arange(31) - 15) * 1.25)
    assert np.array_equal(phi[:, 15], np.abs(np.arange(21) - 10) * 0.5)
    # the first diagonal neighbour: both axes upwind with minima (dx, dy)
    want = _printed_alg12(0.5, 1.25, 1.25, 0.5, 1.0)  # a_x = phi(y+-1) = dy, a_y = phi(x+-1) = dx
    assert phi[11, 16] == pytest.approx(want, rel=1e-15)


def test_strip_is_the_sum_of_spacing_over_speed():
    F = np.exp(R.uniform(-1, 1, size=(1, 40)))
    phi = oracle.fmm(F, 1.0, [0], spacing=(3.0, 0.3))
    want = np.concatenate([[0.0], np.cumsum(0.3 / F[0, 1:])])
    assert np.allclose(phi[0], want, rtol=1e-14, atol=0)


@pytest.mark.parametrize("nd,seed", [(2, 1), (2, 2), (3, 3), (3, 4)])
def test_fmm_equals_sweeping_and_fim(nd, seed):
    r = np.random.default_rng(seed)
    dims = tuple(int(v) for v in r.integers(4, 18 if nd == 2 else 9, size=nd))
    F = np.exp(r.uniform(-1, 1, size=dims))
    F[r.random(dims) < 0.1] = 0.0
    n = F.size
    src = r.choice(n, size=3, replace=False)
    sp = tuple(r.uniform(0.2, 2.0, size=nd))
    ref = oracle.fmm(F, 1.0, src, spacing=sp)
    fsm, _ = oracle.fsm(F, 1.0, src, spacing=sp)
    fim, _ = oracle.fim(F, 1.0, src, spacing=sp)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(fsm)) and np.array_equal(fin, np.isfinite(fim))
    assert np.max(np.abs(fsm[fin] - ref[fin])) <= 1e-13 * ref[fin].max()
    assert np.max(np.abs(fim[fin] - ref[fin])) <= 1e-13 * ref[fin].max()
    # fixed point of the anisotropic local solve
    g = oracle.apply_local(F, 1.0, ref, spacing=sp)
    m = fin & ~np.isin(np.arange(n).reshape(dims), src)
    assert np.max(np.abs(g[m] - ref[m])) <= 1e-13 * ref[fin].max()


def test_scaling_with_the_spacing():
    F = np.exp(R.uniform(-1, 1, size=(15, 12, 9)))
    a = oracle.fmm(F, 1.0, [5], spacing=(0.5, 1.0, 2.0))
    b = oracle.fmm(F, 1.0, [5], spacing=(1.5, 3.0, 6.0))
    assert np.allclose(b, 3.0 * a, rtol=1e-13, atol=0)


def test_adjoint_finite_differences_and_euler():
    r = np.random.default_rng(77)
    dims = (14, 11)
    F = np.exp(r.uniform(-0.5, 0.5, size=dims))
    sp = (0.6, 1.4)
    src = [0]
    g = np.zeros(dims)
    g[-1, :] = r.uniform(0.5, 1.5, size=dims[1])
    phi = oracle.fmm(F, 1.0, src, spacing=sp)
    d = oracle.adjoint(F, 1.0, src, phi, g, spacing=sp)
    L = float((g * phi).sum())
    assert float((F * d).sum()) == pytest.approx(-L, rel=1e-12)
    checked = 0
    for c in r.choice(np.arange(1, F.size), size=20, replace=False):
        dF = 1e-6 * F.flat[c]
        Fp = F.copy(); Fp.flat[c] += dF
        Fm = F.copy(); Fm.flat[c] -= dF
        pp, pm = oracle.fmm(Fp, 1.0, src, spacing=sp), oracle.fmm(Fm, 1.0, src, spacing=sp)
        if not np.array_equal(H.upwind_signature(pp), H.upwind_signature(pm)):
            continue
        fd = float(((pp - pm) * g).sum() / (2 * dF))
        assert d.flat[c] == pytest.approx(fd, rel=1e-5, abs=1e-8 * np.abs(d).max())
        checked += 1
    assert checked >= 10
