"""Pins of the checks in tests/oracle_checks.py, on the CPU.

The float32 adjoint bound is exercised with a plain float32 restatement of
the adjoint (pull form, nodes in decreasing phi): its error against the
float64 oracle must stay inside the bound at every node, and an error of a
few parts in 10^5 planted in one coefficient must break it.  The fixed-point
distance is exercised with the oracle's float32 Algorithm 2 emulation (a
float32 fixed point) and with a value moved by 16 ulp."""

import numpy as np
import pytest

import oracle
import workloads as W
from tests.oracle_checks import U32, chain_bound, fixed_point_ulps, fp32_adjoint_bound


def _adjoint_f32(F, h, sources, phi, g, plant=None):
    """dL/dF in float32 arithmetic: c_ik = w_ik / W_i, lambda_j = g_j + sum of
    c_ij lambda_i over the nodes i that j is upwind of, dL/dF = D lambda.
    plant = (node, factor) scales one coefficient of that node."""
    f = F.astype(np.float32).ravel()
    p = phi.astype(np.float32).ravel()
    gg = g.astype(np.float32).ravel()
    shape = F.shape
    nd = F.ndim
    strides = [int(np.prod(shape[k + 1:])) for k in range(nd)]
    src = set(int(s) for s in np.ravel(sources))
    h32 = np.float32(h)
    coef = {}   # i -> list of (j, c)
    D = np.zeros(p.size, dtype=np.float32)
    for i in range(p.size):
        if i in src or not np.isfinite(p[i]) or not f[i] > 0:
            continue
        coord = np.unravel_index(i, shape)
        ups, ws = [], []
        for k in range(nd):
            best, v = -1, np.float32(np.inf)
            if coord[k] > 0 and p[i - strides[k]] < v:
                best, v = i - strides[k], p[i - strides[k]]
            if coord[k] + 1 < shape[k] and p[i + strides[k]] < v:
                best, v = i + strides[k], p[i + strides[k]]
            if best >= 0 and v < p[i]:
                ups.append(best)
                ws.append(np.float32(p[i] - v))
        if not ups:
            continue
        W_ = np.float32(0)
        for w in ws:
            W_ = np.float32(W_ + w)
        cs = [np.float32(w / W_) for w in ws]
        if plant is not None and plant[0] == i:
            cs[0] = np.float32(cs[0] * plant[1])
        coef[i] = list(zip(ups, cs))
        Hh = np.float32(h32 / f[i])
        D[i] = -np.float32(np.float32(Hh * Hh) / np.float32(f[i] * W_))
    pulls = {}  # j -> list of (i, c_ij)
    for i, lst in coef.items():
        for j, c in lst:
            pulls.setdefault(j, []).append((i, c))
    lam = gg.copy()
    order = np.argsort(-np.where(np.isfinite(p), p, -np.inf), kind="stable")
    for j in order:
        v = gg[j]
        for i, c in pulls.get(int(j), []):
            v = np.float32(v + np.float32(c * lam[i]))
        lam[j] = v
    return (D * lam).reshape(shape).astype(np.float64)


def _case(P, seed):
    phi = oracle.fmm(P.F.astype(np.float32).astype(np.float64), P.h, P.sources).astype(np.float32)
    r = np.random.default_rng(seed)
    g = np.zeros(P.F.shape)
    fin = np.flatnonzero(np.isfinite(phi.ravel()))
    pick = r.choice(fin, size=min(10, fin.size), replace=False)
    g.flat[pick] = r.uniform(-2, 2, size=pick.size)
    return phi, g


@pytest.mark.parametrize("P", [W.lognormal_2d(24, seed=5), W.layered_3d(9, n_receivers=6),
                               W.random_problem(31, 2, 20, zero_frac=0.1)], ids=lambda P: P.name)
def test_fp32_adjoint_within_bound(P):
    phi, g = _case(P, 3)
    Fq = P.F.astype(np.float32).astype(np.float64)
    got = _adjoint_f32(P.F, P.h, P.sources, phi, g)
    want = oracle.adjoint(Fq, P.h, P.sources, phi.astype(np.float64), g)
    bound = fp32_adjoint_bound(Fq, P.h, P.sources, phi, g)
    err = np.abs(got - want)
    assert np.all(err <= bound + 1e-300)
    # not vacuous: the bound is a small multiple of u relative to the gradient
    assert bound.max() <= 1e4 * U32 * np.abs(want).max()


def test_fp32_adjoint_bound_catches_planted_coefficient_errors():
    """One coefficient of a node scaled by 1 + 5e-5, dropped (0) or negated:
    it changes lambda of the node's upwind neighbour (nothing when that is a
    source, whose gradient is 0).  Over the ten nodes with the largest
    gradient, most such errors break the bound."""
    P = W.lognormal_2d(24, seed=5)
    phi, g = _case(P, 3)
    Fq = P.F.astype(np.float32).astype(np.float64)
    want = oracle.adjoint(Fq, P.h, P.sources, phi.astype(np.float64), g)
    bound = fp32_adjoint_bound(Fq, P.h, P.sources, phi, g)
    top = np.argsort(-np.abs(want.ravel()))[:10]
    for fac, need in ((1 + 5e-5, 5), (0.0, 7), (-1.0, 7)):
        caught = sum(int(np.any(np.abs(_adjoint_f32(P.F, P.h, P.sources, phi, g,
                                                    plant=(int(i), np.float32(fac))) - want) > bound))
                     for i in top)
        assert caught >= need, (fac, caught)


def test_fixed_point_ulps_of_a_float32_fixed_point():
    P = W.lognormal_2d(64, seed=2)
    phi, _ = oracle.ifim(P.F, P.h, P.sources, dtype=np.float32)
    r = fixed_point_ulps(P.F, P.h, phi, P.sources)
    assert r.max() <= 4.0
    moved = phi.copy()
    k = np.flatnonzero(np.isfinite(moved.ravel()) & (moved.ravel() > 0.5 * np.nanmax(moved)))[0]
    moved.flat[k] = np.float32(moved.flat[k]) + 16 * np.spacing(np.float32(moved.flat[k]))
    assert fixed_point_ulps(P.F, P.h, moved, P.sources).max() >= 8.0


def test_fp32_adjoint_bound_covers_underflow():
    """A loss gradient scaled into float32's subnormal range: the float32
    adjoint then rounds to multiples of 2^-149, an absolute error the relative
    part of the bound cannot cover; the underflow floor does, and stays far
    below any normal-range gradient."""
    P = W.lognormal_2d(24, seed=5)
    phi, g = _case(P, 3)
    g = g * 2.0 ** -135
    Fq = P.F.astype(np.float32).astype(np.float64)
    got = _adjoint_f32(P.F, P.h, P.sources, phi, g)
    want = oracle.adjoint(Fq, P.h, P.sources, phi.astype(np.float64), g)
    bound = fp32_adjoint_bound(Fq, P.h, P.sources, phi, g)
    err = np.abs(got - want)
    assert np.all(err <= bound + 1e-300)
    relative_only = U32 * 100.0 * np.abs(want)
    assert np.any(err > relative_only), "expected subnormal rounding beyond any relative bound"
    assert bound.max() <= 1e-30


@pytest.mark.parametrize("P", [W.paper_example(1, 300), W.paper_example(3, 200), W.lognormal_2d(96, seed=4),
                               W.maze_3d(24)], ids=lambda P: P.name)
def test_chain_bound_holds_for_the_float32_emulation(P):
    """The oracle's float32 emulation of Algorithm 2 (a float32 fixed point)
    stays within chain_bound of the float64 fixed point; a value lowered by
    a thousandth of max phi (a wrong but locally consistent node would need
    its neighbours to follow) shows up as a residual far above it."""
    phi, _ = oracle.ifim(P.F, P.h, P.sources, dtype=np.float32, values=P.source_values)
    ref = oracle.fmm(P.F.astype(np.float32).astype(np.float64), P.h, P.sources, values=P.source_values)
    err = float(np.max(np.abs(phi.astype(np.float64)[np.isfinite(ref)] - ref[np.isfinite(ref)])))
    b = chain_bound(P.F.astype(np.float32), P.h, P.sources, phi, P.source_values)
    assert err <= b
    assert b <= 1e-2 * float(np.max(ref[np.isfinite(ref)]))
    bad = phi.copy()
    fin = np.flatnonzero(np.isfinite(bad.ravel()))
    k = fin[np.argmax(bad.ravel()[fin])]
    bad.flat[k] = np.float32(bad.flat[k] - 1e-3 * np.max(bad.ravel()[fin]))
    assert fixed_point_ulps(P.F.astype(np.float32), P.h, bad, P.sources).max() > 100.0
