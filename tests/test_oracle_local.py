"""Pins of the oracle's local solver (Eq 4 / Eq 6; Algorithms 1.1 and 1.3).

The expected values come from hand-derived closed forms (tests/golden), from
bisection on the defining residual, and from properties of the exact root.
"""

import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "local_solver_closed_forms.csv")


def _cases():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            a1, a2, a3, H, expr, note = line.split(";", 5)
            a = [float(v) for v in (a1, a2, a3) if v != ""]
            rows.append((a, float(H), expr, note))
    return rows


CASES = _cases()


def _eval(expr):
    return float(eval(expr, {"__builtins__": {}}, {"sqrt": math.sqrt, "inf": math.inf}))


@pytest.mark.parametrize("a,H,expr,note", CASES, ids=[c[3] for c in CASES])
def test_closed_form(a, H, expr, note):
    want = _eval(expr)
    got = oracle.godunov(a, H)
    if math.isinf(want):
        assert math.isinf(got)
        return
    assert got == pytest.approx(want, rel=4e-16, abs=0.0)
    assert oracle.godunov_bisect(a, H) == pytest.approx(want, rel=1e-15, abs=0.0)
    got32 = float(oracle.godunov_f(a, H))
    assert got32 == pytest.approx(want, rel=4 * 2.0 ** -24)
    # permutation invariance of the inputs
    assert oracle.godunov(list(reversed(a)), H) == got


def _rand_vectors(seed, n):
    r = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        m = int(r.integers(2, 4))
        base = float(r.choice([0.0, 1.0, 50.0, 1e3]))
        H = float(np.exp(r.uniform(np.log(1e-3), np.log(1e3))))
        a = base + r.uniform(0, 1.5 * H, size=m)
        if r.random() < 0.2:
            a[int(r.integers(0, m))] = np.inf
        out.append((list(a), H))
    return out


def test_random_matches_bisection():
    for a, H in _rand_vectors(1, 3000):
        got = oracle.godunov(a, H)
        ref = oracle.godunov_bisect(a, H)
        assert got == pytest.approx(ref, rel=2e-15, abs=1e-300), (a, H)


def test_random_satisfies_godunov_equation():
    # sum_k ((phi - a_k)^+)^2 = H^2  (Eq 4 / Eq 6 with Delta = h, H = h/F)
    for a, H in _rand_vectors(2, 3000):
        phi = oracle.godunov(a, H)
        s = sum(max(phi - ak, 0.0) ** 2 for ak in a if math.isfinite(ak))
        # rounding of phi perturbs each upwind difference by ~eps*|phi|
        scale = H * H + 2 * abs(phi) * sum(phi - ak for ak in a if math.isfinite(ak) and ak < phi)
        assert abs(s - H * H) <= 16 * 2.2e-16 * scale, (a, H, phi)


def test_bounds_and_monotonicity():
    r = np.random.default_rng(3)
    for a, H in _rand_vectors(4, 1500):
        phi = oracle.godunov(a, H)
        a1 = min(a)
        m = len(a)
        assert a1 + H / math.sqrt(m) * (1 - 1e-14) <= phi <= a1 + H * (1 + 1e-15)
        # raising one neighbour never lowers the update; lowering never raises it
        k = int(r.integers(0, m))
        if math.isfinite(a[k]):
            up = list(a)
            up[k] += float(r.uniform(0, H))
            assert oracle.godunov(up, H) >= phi
        # larger H (slower speed) never lowers the update
        assert oracle.godunov(a, H * 1.5) >= phi


def test_infinite_cases():
    assert math.isinf(oracle.godunov([np.inf, np.inf], 1.0))
    assert math.isinf(oracle.godunov([0.0, 1.0], np.inf))
    assert math.isinf(oracle.godunov([np.inf, np.inf, np.inf], 1.0))
    assert oracle.godunov([np.inf, 2.0, np.inf], 0.5) == 2.5


def _paper_alg11_literal(a, b, delta_over_f):
    """Algorithm 1.1 exactly as printed (sqrt(2) threshold)."""
    if abs(a - b) > math.sqrt(2) * delta_over_f:
        return min(a, b) + delta_over_f
    return 0.5 * (a + b + math.sqrt(2 * delta_over_f ** 2 - (a - b) ** 2))


def test_printed_alg11_threshold_does_not_solve_eq4():
    """Reading of Algorithm 1.1: the printed threshold switches to the one-sided
    update too late; at (0, 1.2, H=1) it returns 0.974..., which violates Eq 4
    (the upwind difference to b would be negative), while the exact solver
    returns 1 and satisfies it."""
    lit = _paper_alg11_literal(0.0, 1.2, 1.0)
    assert lit == pytest.approx(0.974165738677394, rel=1e-14)
    # Eq 4 residual of the printed value: only the x-term is upwind.
    assert abs(max(lit - 0.0, 0) ** 2 + max(lit - 1.2, 0) ** 2 - 1.0) > 0.05
    exact = oracle.godunov([0.0, 1.2], 1.0)
    assert exact == 1.0
    # where both branches are valid the printed two-sided formula agrees
    assert _paper_alg11_literal(0.0, 0.5, 1.0) == pytest.approx(oracle.godunov([0.0, 0.5], 1.0), rel=1e-15)


def test_float32_solver_close_to_float64():
    for a, H in _rand_vectors(5, 2000):
        a32 = [float(np.float32(v)) for v in a]
        H32 = float(np.float32(H))
        ref = oracle.godunov(a32, H32)
        got = float(oracle.godunov_f(a32, H32))
        if math.isinf(ref):
            assert math.isinf(got)
        else:
            assert got == pytest.approx(ref, rel=8 * 2.0 ** -24), (a, H)
