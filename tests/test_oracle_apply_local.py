"""Pins of the oracle's whole-grid local solve G_i(phi) (Eq 4 / Eq 6 at every
node; isotropic spacing).  This is the function the GPU's apply-local entry
point must match bit for bit, so it is pinned on its own:

* hand-computed grids whose every entry follows from Eq 4 / Eq 6 by hand
  (asymmetric values, so a swapped axis, a one-sided neighbour read or a
  dropped out-of-grid rule changes some entry);
* barriers (F = 0) and all-infinite neighbourhoods give +inf;
* on the fast-marching solution it returns that solution at every finite
  non-source node (the solution is the fixed point of the system);
* on a 1D strip it reproduces the one-sided sums.
"""

import math

import numpy as np
import pytest

import oracle
import workloads as W

INF = math.inf
R2 = math.sqrt(2.0)


def test_hand_computed_2d():
    # phi, F and h chosen so that every node exercises a different case
    phi = np.array([[0.0, 1.0, 2.0],
                    [1.0, INF, INF],
                    [2.0, INF, INF]])
    F = np.array([[1.0, 1.0, 1.0],
                  [1.0, 0.5, 1.0],
                  [1.0, 1.0, 0.0]])
    got = oracle.apply_local(F, 1.0, phi)
    want = np.array([
        # (0,0): a = (1, 1), H = 1, two-sided: 1 + sqrt(2)/2
        # (0,1): a_y = +inf, a_x = min(0, 2) = 0 -> one-sided 1
        # (0,2): a_y = +inf, a_x = 1 -> 2
        [1.0 + R2 / 2.0, 1.0, 2.0],
        # (1,0): a_y = min(0, 2) = 0, a_x = +inf -> 1
        # (1,1): a = (1, 1), H = 2: 1 + sqrt(8)/2 = 1 + sqrt(2)
        # (1,2): a_y = min(2, +inf) = 2, a_x = +inf -> 3
        [1.0, 1.0 + R2, 3.0],
        # (2,0): a_y = 1, a_x = +inf -> 2
        # (2,1): a_y = +inf, a_x = min(2, +inf) = 2 -> 3
        # (2,2): F = 0 -> +inf
        [2.0, 3.0, INF],
    ])
    assert np.array_equal(np.isinf(got), np.isinf(want))
    fin = np.isfinite(want)
    np.testing.assert_allclose(got[fin], want[fin], rtol=2e-16, atol=0)


def test_hand_computed_2d_one_sided_branch_and_spacing():
    # a = (0, 1.5), H = 1: the one-sided value 1 does not exceed 1.5, so the
    # second axis is not upwind; with h = 2 the two-sided root
    # (1.5 + sqrt(2 * 4 - 1.5^2)) / 2 is taken instead.
    phi = np.array([[INF, 0.0, INF],
                    [1.5, INF, INF]])
    F = np.ones_like(phi)
    g1 = oracle.apply_local(F, 1.0, phi)
    assert g1[1, 1] == 1.0
    g2 = oracle.apply_local(F, 2.0, phi)
    assert g2[1, 1] == pytest.approx((1.5 + math.sqrt(8.0 - 2.25)) / 2.0, rel=2e-16)
    # node (0,0): a_y = 1.5 (below), a_x = 0 (right): the same pair, so
    # one-sided 1 with h = 1 and the same two-sided root with h = 2
    assert g1[0, 0] == 1.0 and g2[0, 0] == g2[1, 1]
    # node (1,2): a_y = +inf, a_x = +inf -> +inf
    assert g1[1, 2] == INF
    # node (0,2): a_y = +inf, a_x = 0 -> h
    assert g1[0, 2] == 1.0


def test_hand_computed_3d():
    # centre node of a 3x3x3 grid with axis minima a = (0, 0, 0.5), H = 1:
    # three-sided root (1 + sqrt(1 - 3 (0.25 - 1))) / 3
    phi = np.full((3, 3, 3), INF)
    phi[0, 1, 1] = 0.0    # axis 0 neighbour (below)
    phi[1, 2, 1] = 0.0    # axis 1 neighbour (after)
    phi[1, 1, 0] = 0.5    # axis 2 neighbour (before)
    F = np.ones_like(phi)
    got = oracle.apply_local(F, 1.0, phi)
    # shifted: b = (0, 0, 0.5) relative to a_1 = 0 -> (S + sqrt(S^2 - 3 (Q - H^2))) / 3
    want = (0.5 + math.sqrt(0.25 - 3.0 * (0.25 - 1.0))) / 3.0
    assert got[1, 1, 1] == pytest.approx(want, rel=4e-16)
    assert got[1, 1, 1] == pytest.approx(0.69371294336139666, rel=4e-16)
    # a node two cells from every finite value sees only +inf
    assert got[2, 0, 2] == INF
    # node (1,1,2): axis 2 neighbour (1,1,1) is +inf, others too -> +inf
    assert got[1, 1, 2] == INF
    # node (0,1,0): axis 0 neighbour (1,1,0) = 0.5, axis 1 +inf, axis 2
    # neighbour (0,1,1) = 0: a = (0, 0.5), two-sided root (0.5 + sqrt(1.75)) / 2
    assert got[0, 1, 0] == pytest.approx(0.91143782776614768, rel=4e-16)
    # node (1,0,1): axis 0 neighbour (0,0,1) +inf, axis 1 neighbour (1,1,1)
    # +inf, axis 2 +inf -> +inf
    assert got[1, 0, 1] == INF
    # the value depends on which axis carries the 0.5: permuting the axes of
    # phi permutes the output
    for perm in [(1, 0, 2), (2, 1, 0), (0, 2, 1)]:
        gp = oracle.apply_local(F, 1.0, np.transpose(phi, perm))
        assert np.array_equal(gp, np.transpose(got, perm))


def test_barriers_and_infinite_neighbourhoods():
    rng = np.random.default_rng(5)
    F = rng.uniform(0.5, 2.0, size=(6, 7))
    F[2, 3] = 0.0
    phi = rng.uniform(0.0, 5.0, size=F.shape)
    got = oracle.apply_local(F, 0.3, phi)
    assert got[2, 3] == INF
    assert np.all(np.isfinite(np.delete(got.ravel(), 2 * 7 + 3)))
    assert np.all(np.isinf(oracle.apply_local(F, 0.3, np.full(F.shape, INF))))


@pytest.mark.parametrize("P", [W.random_problem(300 + s, 2, 24, zero_frac=0.05) for s in range(4)]
                         + [W.random_problem(400 + s, 3, 10, zero_frac=0.05) for s in range(3)],
                         ids=lambda P: "x".join(map(str, P.F.shape)))
def test_fixed_point_of_fast_marching(P):
    """fmm computes each node from its accepted neighbours only; apply_local
    reads every neighbour.  At the solution the two agree on every finite
    non-source node (to the last bit on these cases; gate 1 ulp)."""
    phi = oracle.fmm(P.F, P.h, P.sources)
    g = oracle.apply_local(P.F, P.h, phi)
    m = np.isfinite(phi)
    m.flat[np.asarray(P.sources)] = False
    assert np.array_equal(np.isfinite(g[m]), np.ones(m.sum(), bool))
    assert np.all(np.abs(g[m] - phi[m]) <= np.spacing(phi[m]))
    # unreachable nodes (walled off by barriers) stay unreachable
    assert np.all(np.isinf(g[np.isinf(phi) & (P.F > 0)]))
    # lowering one value never raises a local value (monotone), and lowering
    # a value that is upwind for a neighbour lowers that neighbour's
    seen = False
    for i in np.flatnonzero(m)[::7][:40]:
        p2 = phi.copy()
        p2.flat[i] *= 0.99
        g2 = oracle.apply_local(P.F, P.h, p2)
        assert np.all(g2 <= g)
        assert g2.flat[i] == g.flat[i]
        seen |= bool(np.any(g2 < g))
    assert seen


def test_one_dimensional_strip():
    rng = np.random.default_rng(11)
    F = rng.uniform(0.2, 3.0, size=(1, 40))
    h = 0.25
    s = 13
    phi = np.zeros_like(F)
    for j in range(s + 1, 40):
        phi[0, j] = phi[0, j - 1] + h / F[0, j]
    for j in range(s - 1, -1, -1):
        phi[0, j] = phi[0, j + 1] + h / F[0, j]
    g = oracle.apply_local(F, h, phi)
    idx = np.arange(40) != s
    np.testing.assert_allclose(g[0, idx], phi[0, idx], rtol=4e-16, atol=0)
    # at the source the local solve returns the nearer neighbour plus its H
    assert g[0, s] == pytest.approx(min(phi[0, s - 1], phi[0, s + 1]) + h / F[0, s], rel=1e-16)


def test_float32_agrees_with_float64_to_rounding():
    P = W.random_problem(77, 3, 12)
    phi = oracle.fmm(P.F, P.h, P.sources)
    g64 = oracle.apply_local(P.F.astype(np.float32), P.h, phi.astype(np.float32))
    g32 = oracle.apply_local(P.F.astype(np.float32), P.h, phi.astype(np.float32), dtype=np.float32)
    fin = np.isfinite(g64)
    assert np.array_equal(fin, np.isfinite(g32))
    assert np.all(np.abs(g32[fin] - g64[fin]) <= 8 * np.spacing(np.abs(g64[fin]).astype(np.float32)))
