"""The paper's own examples (Results: Examples 1, 2, 3, 5) on the oracle.

What the paper states about them, checked at 200^2:
  * all methods give the same solution (FMM, FSM, FIM and the improved method);
  * Example 1 (one circle, F = 1) needs no remedy: the update step alone is
    exact;
  * Examples 2 and 5 (and 3) leave errors after the update step that the
    remedy step removes.
Plus the continuum limit of Example 1: the arrival time approaches the
distance to the circle with first-order error in h."""

import numpy as np
import pytest

import oracle
import workloads as W


def _solve_all(P):
    ref = oracle.fmm(P.F, P.h, P.sources, values=P.source_values)
    upd, _ = oracle.ifim(P.F, P.h, P.sources, values=P.source_values, skip_remedy=True)
    full, st = oracle.ifim(P.F, P.h, P.sources, values=P.source_values)
    fim, _ = oracle.fim(P.F, P.h, P.sources, values=P.source_values)
    return ref, upd, full, st, fim


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_all_methods_agree(k):
    P = W.paper_example(k, 200, dtype=np.float64)
    ref, _, full, _, fim = _solve_all(P)
    assert np.all(np.isfinite(ref))
    assert np.array_equal(full, ref) and np.array_equal(fim, ref)
    fsm, _ = oracle.fsm(P.F, P.h, P.sources, values=P.source_values)
    assert np.max(np.abs(fsm - ref)) <= 1e-13 * ref.max()


def test_example1_needs_no_remedy():
    P = W.paper_example(1, 200, dtype=np.float64)
    ref, upd, _, st, _ = _solve_all(P)
    assert np.array_equal(upd, ref)
    assert st["remedy_initial"] == 0 and st["evals_remedy"] == 0


@pytest.mark.parametrize("k", [2, 3, 5])
def test_examples_with_remedy(k):
    P = W.paper_example(k, 200, dtype=np.float64)
    ref, upd, full, st, _ = _solve_all(P)
    assert np.any(upd > ref * (1 + 1e-12)) and np.all(upd >= ref)
    assert st["remedy_initial"] > 0
    assert np.array_equal(full, ref)


def test_example1_converges_to_the_distance():
    """F = 1: the exact arrival time is |dist - 3|; the first-order scheme's
    error shrinks with h."""
    errs = []
    for n in (101, 201, 401):
        P = W.paper_example(1, n, dtype=np.float64)
        phi = oracle.fmm(P.F, P.h, P.sources, values=P.source_values)
        h, ys, xs = 20.0 / (n - 1), *np.meshgrid(np.linspace(-10, 10, n), np.linspace(-10, 10, n), indexing="ij")
        exact = np.abs(np.sqrt(xs ** 2 + ys ** 2) - 3.0)
        errs.append(np.max(np.abs(phi - exact)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.6 * errs[1]
