"""Pins of the oracle's grid solvers against closed forms, brute force and
invariants of the discrete Godunov system (Eq 4 / Eq 6), and of the serial
Algorithm 2 emulation against the paper's behavioural claims."""

import math

import numpy as np
import pytest

import oracle
import workloads as W
from tests import helpers as H


def _random_cases(n2=12, n3=8, zero_frac=0.0, base=100):
    cases = []
    for s in range(n2):
        cases.append(W.random_problem(base + s, 2, 20, zero_frac=zero_frac))
    for s in range(n3):
        cases.append(W.random_problem(base + 1000 + s, 3, 8, zero_frac=zero_frac))
    return cases


def test_constant_speed_axis_values_exact():
    """F = 1, point source: along the grid lines through the source the update
    is one-sided, so phi = |offset| * h exactly; diagonal neighbour solves
    2 (phi - 1)^2 = 1."""
    P = W.tiny_constant()
    phi = oracle.fmm(P.F, P.h, P.sources)
    assert phi[32, 32] == 0.0
    for k in range(-32, 32):
        assert phi[32, 32 + k] == abs(k)
        assert phi[32 + k, 32] == abs(k)
    assert phi[33, 33] == pytest.approx(1 + 1 / math.sqrt(2), rel=1e-16)
    # global bounds for constant F: |d|_1 h / sqrt(2) <= phi <= |d|_1 h
    yy, xx = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
    l1 = np.abs(yy - 32) + np.abs(xx - 32)
    assert np.all(phi <= l1 + 1e-12)
    assert np.all(phi >= l1 / math.sqrt(2) - 1e-12)
    assert H.equation_residual(P.F, P.h, phi, P.sources) < 1e-13
    assert H.causality_ok(P.F, phi, P.sources)
    # eight-fold symmetry of the stencil around the source
    sub = phi[1:, 1:]  # centred 63x63 window
    assert np.array_equal(sub, sub[::-1, :]) and np.array_equal(sub, sub.T)


def test_constant_speed_3d_axis_and_diagonal():
    dims = (9, 9, 9)
    F = np.ones(dims)
    src = [W.flat_index(dims, (4, 4, 4))]
    phi = oracle.fmm(F, 1.0, src)
    for k in range(-4, 5):
        assert phi[4, 4, 4 + k] == abs(k)
    assert phi[5, 5, 4] == pytest.approx(1 + 1 / math.sqrt(2), rel=1e-16)
    assert H.equation_residual(F, 1.0, phi, src) < 1e-13
    assert H.local_bounds_ok(F, 1.0, phi, src)


def test_one_dimensional_strip_exact():
    """On a (1, n) strip every update is one-sided: phi_i is the sum of h/F_j
    over the path from the source, excluding the source, including i."""
    r = np.random.default_rng(7)
    for n in (2, 7, 40):
        F = np.exp(r.uniform(-3, 3, size=(1, n)))
        h = float(r.uniform(0.1, 3.0))
        s = int(r.integers(0, n))
        phi = oracle.fmm(F, h, [s])
        Hc = h / F[0]
        for i in range(n):
            lo, hi = (s, i) if i >= s else (i, s)
            path = range(lo + 1, hi + 1) if i >= s else range(lo, hi)
            want = 0.0
            for j in path:
                want += Hc[j]
            assert phi[0, i] == pytest.approx(want, rel=1e-14, abs=0)


def test_source_values_and_duplicates():
    F = np.ones((1, 10))
    # two sources with values; duplicate index keeps the minimum value
    phi = oracle.fmm(F, 1.0, [2, 7, 7], values=[0.5, 3.0, 1.0])
    want = np.minimum(0.5 + np.abs(np.arange(10) - 2), 1.0 + np.abs(np.arange(10) - 7))
    assert np.array_equal(phi[0], want)


@pytest.mark.parametrize("P", _random_cases(), ids=lambda P: P.name)
def test_fmm_equals_fast_sweeping(P):
    """Brute force: Gauss-Seidel with the 2^d orderings of the fast sweeping
    method, repeated until a full pass changes nothing, reaches the same
    fixed point."""
    phi = oracle.fmm(P.F, P.h, P.sources)
    ref, _ = oracle.fsm(P.F, P.h, P.sources)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(phi))
    m = np.nanmax(np.where(fin, ref, np.nan)) if fin.any() else 1.0
    assert np.max(np.abs(phi[fin] - ref[fin])) <= 1e-14 * max(m, 1e-300)


@pytest.mark.parametrize("P", _random_cases(4, 2, base=300), ids=lambda P: P.name)
def test_fmm_equals_bisection_sweeping(P):
    """Same brute force with the local solve done by bisection on the Godunov
    residual, i.e. without the closed-form quadratic."""
    phi = oracle.fmm(P.F, P.h, P.sources)
    ref, _ = oracle.fsm(P.F, P.h, P.sources, bisect=True)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(phi))
    m = ref[fin].max()
    assert np.max(np.abs(phi[fin] - ref[fin])) <= 1e-12 * max(m, 1e-300)


@pytest.mark.parametrize("P", _random_cases(8, 6, zero_frac=0.25, base=500), ids=lambda P: P.name)
def test_barriers_and_unreachable(P):
    """F = 0 cells are barriers (Eq 8): nodes cut off from every source stay
    +inf, everything else is finite and satisfies the discrete equation."""
    phi = oracle.fmm(P.F, P.h, P.sources)
    unreach = H.unreachable_mask(P.F, P.sources)
    barrier = (P.F == 0)
    src = np.zeros(P.F.shape, dtype=bool)
    src.flat[P.sources] = True
    want_inf = (unreach | barrier) & ~src
    assert np.array_equal(~np.isfinite(phi), want_inf)
    assert H.equation_residual(P.F, P.h, phi, P.sources) < 1e-12
    assert H.causality_ok(P.F, phi, P.sources)
    ref, _ = oracle.fsm(P.F, P.h, P.sources)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(phi))
    if fin.any():
        assert np.max(np.abs(phi[fin] - ref[fin])) <= 1e-14 * ref[fin].max() + 1e-300


@pytest.mark.parametrize("P", _random_cases(6, 4, base=700), ids=lambda P: P.name)
def test_invariants(P):
    phi = oracle.fmm(P.F, P.h, P.sources)
    assert H.equation_residual(P.F, P.h, phi, P.sources) < 1e-12
    assert H.causality_ok(P.F, phi, P.sources)
    assert H.local_bounds_ok(P.F, P.h, phi, P.sources)
    # scaling: phi(2F) = phi(F)/2, phi(2h) = 2 phi(h) (powers of two: exact)
    assert np.array_equal(oracle.fmm(2 * P.F, P.h, P.sources), phi / 2)
    assert np.array_equal(oracle.fmm(P.F, 2 * P.h, P.sources), phi * 2)
    # F-monotonicity: a faster medium never arrives later
    r = np.random.default_rng(1)
    Fp = P.F * np.exp(r.uniform(0, 1, size=P.F.shape))
    assert np.all(oracle.fmm(Fp, P.h, P.sources) <= phi * (1 + 1e-14))
    # source union: adding a source never raises a value
    extra = np.append(P.sources, int(r.integers(0, P.F.size)))
    assert np.all(oracle.fmm(P.F, P.h, extra) <= phi)


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_symmetry(seed):
    """Axis flips and transposes of (F, sources) commute with the solve."""
    P = W.random_problem(seed, 3, 7)
    phi = oracle.fmm(P.F, P.h, P.sources)
    coords = np.stack(np.unravel_index(P.sources, P.F.shape), 1)
    # flip axis 1
    Ff = P.F[:, ::-1, :].copy()
    cf = coords.copy()
    cf[:, 1] = P.F.shape[1] - 1 - cf[:, 1]
    sf = np.ravel_multi_index(cf.T, Ff.shape)
    assert np.array_equal(oracle.fmm(Ff, P.h, sf)[:, ::-1, :], phi)
    # transpose (2, 0, 1)
    Ft = np.ascontiguousarray(P.F.transpose(2, 0, 1))
    ct = coords[:, [2, 0, 1]]
    st = np.ravel_multi_index(ct.T, Ft.shape)
    assert np.array_equal(oracle.fmm(Ft, P.h, st), phi.transpose(2, 0, 1))


# ---------------------------------------------------------------------------
# Algorithm 2 emulation
# ---------------------------------------------------------------------------

def _workload_cases():
    return [
        W.lognormal_2d(48, dtype=np.float64),
        W.lognormal_2d(64, seed=5, dtype=np.float64),
        W.Problem("maze2d", W.maze_field((64, 64), 9, free_coord=(0, 0), dtype=np.float64), 1.0,
                  np.array([0])),
        W.maze_3d(24, dtype=np.float64),
        W.random_problem(42, 2, 30, zero_frac=0.1),
        W.random_problem(43, 3, 10, zero_frac=0.1),
    ]


@pytest.mark.parametrize("P", _workload_cases() + _random_cases(4, 4, base=900), ids=lambda P: P.name)
def test_ifim_reaches_the_fixed_point(P):
    """Algorithm 2 run to completion (update, detection, remedy) yields the
    same solution as fast marching (the paper reports identical solutions for
    all four methods in every example)."""
    ref = oracle.fmm(P.F, P.h, P.sources)
    phi, st = oracle.ifim(P.F, P.h, P.sources)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(phi))
    if fin.any():
        assert np.max(np.abs(phi[fin] - ref[fin])) <= 1e-14 * ref[fin].max() + 1e-300
    assert st["evals_detect"] == P.F.size - len(np.unique(P.sources))


def test_ifim_constant_speed_single_source_needs_no_remedy():
    """Example 1's observation: a single front at constant speed is already
    exact after the update step; each node converges on its second
    evaluation."""
    P = W.tiny_constant()
    ref = oracle.fmm(P.F, P.h, P.sources)
    phi2, st2 = oracle.ifim(P.F, P.h, P.sources, eps=P.eps, skip_remedy=True)
    assert np.array_equal(phi2, ref)
    phi, st = oracle.ifim(P.F, P.h, P.sources, eps=P.eps)
    assert np.array_equal(phi, ref)
    n = P.F.size
    assert st["evals_step2"] == 2 * (n - 1)
    assert st["remedy_initial"] == 0 and st["evals_remedy"] == 0
    assert st["step2_iters"] == 128  # two iterations per Manhattan layer (64 layers)


def test_ifim_two_fronts_need_remedy():
    """Example 2's observation: with two sources the update step leaves errors
    which the remedy step removes."""
    dims = (64, 64)
    F = np.ones(dims)
    src = [W.flat_index(dims, (10, 50)), W.flat_index(dims, (50, 10))]
    ref = oracle.fmm(F, 1.0, src)
    phi2, _ = oracle.ifim(F, 1.0, src, skip_remedy=True)
    assert np.any(phi2 > ref)        # update step leaves overestimates
    assert np.all(phi2 >= ref)       # ... and never underestimates
    phi, st = oracle.ifim(F, 1.0, src)
    assert np.array_equal(phi, ref)
    assert st["remedy_initial"] > 0


def test_ifim_variable_speed_needs_remedy():
    """Example 5's observation for a variable speed field."""
    P = W.lognormal_2d(64, dtype=np.float64)
    ref = oracle.fmm(P.F, P.h, P.sources)
    phi2, _ = oracle.ifim(P.F, P.h, P.sources, skip_remedy=True)
    assert np.any(phi2 > ref * (1 + 1e-12)) and np.all(phi2 >= ref)
    phi, _ = oracle.ifim(P.F, P.h, P.sources)
    assert np.array_equal(phi, ref)


def test_ifim_float32_within_tolerance():
    P = W.lognormal_2d(128)
    ref = oracle.fmm(P.F.astype(np.float64), P.h, P.sources)
    phi, _ = oracle.ifim(P.F, P.h, P.sources, dtype=np.float32)
    assert np.max(np.abs(phi - ref)) <= 1e-5 * ref.max()


def test_ifim_iteration_cap_reported():
    P = W.lognormal_2d(32, dtype=np.float64)
    with pytest.raises(RuntimeError):
        oracle.ifim(P.F, P.h, P.sources, max_iters=3)


# ---------------------------------------------------------------------------
# FIM (Section 2.3), the method the improved variant is compared against
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("P", _workload_cases() + _random_cases(4, 4, base=950), ids=lambda P: P.name)
def test_fim_reaches_the_fixed_point(P):
    """FIM's neighbour check re-activates every node a converged neighbour
    would lower, so it ends at the same fixed point as fast marching and as
    the improved method (the paper compares their run times on identical
    solutions)."""
    ref = oracle.fmm(P.F, P.h, P.sources)
    phi, st = oracle.fim(P.F, P.h, P.sources)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(phi))
    if fin.any():
        assert np.max(np.abs(phi[fin] - ref[fin])) <= 1e-14 * ref[fin].max() + 1e-300
    phi_i, _ = oracle.ifim(P.F, P.h, P.sources)
    assert np.array_equal(np.isfinite(phi_i), fin)
    if fin.any():
        assert np.max(np.abs(phi[fin] - phi_i[fin])) <= 1e-14 * ref[fin].max() + 1e-300


def test_fim_checks_neighbours_during_the_update():
    """Section 3.3: FIM evaluates the neighbours of every converged node inside
    the update, work the improved method's update step leaves out.  At
    constant speed from one source both are exact without any remedy, and
    FIM's check evaluations exceed the improved method's whole detection
    pass."""
    P = W.tiny_constant()
    ref = oracle.fmm(P.F, P.h, P.sources)
    phi_f, sf = oracle.fim(P.F, P.h, P.sources, eps=P.eps)
    phi_i, si = oracle.ifim(P.F, P.h, P.sources, eps=P.eps)
    assert np.array_equal(phi_f, ref) and np.array_equal(phi_i, ref)
    n = P.F.size
    assert sf["evals_check"] > si["evals_detect"] == n - 1
    assert sf["evals_update"] >= n - 1          # every reachable node is updated at least once
    assert si["evals_remedy"] == 0


def test_fim_barrier_and_unreachable():
    """A node behind a wall of F = 0 is never activated (+inf); a source on a
    barrier cell still spreads to its passable neighbours."""
    F = np.ones((24, 24))
    F[:, 12] = 0.0
    F[5, 5] = 0.0
    phi, _ = oracle.fim(F, 1.0, [5 * 24 + 5])
    assert np.all(np.isinf(phi[:, 12:]))
    assert np.array_equal(phi, oracle.fmm(F, 1.0, [5 * 24 + 5]))


def test_fim_iteration_cap_reported():
    P = W.lognormal_2d(32, dtype=np.float64)
    with pytest.raises(RuntimeError):
        oracle.fim(P.F, P.h, P.sources, max_iters=3)
