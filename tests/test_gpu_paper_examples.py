"""The paper's Examples 1, 2, 3 and 5 on the GPU: every schedule against the
oracle's fast marching solution (float32 gate), and the paper's observation
on the update step: with synchronous reads (the serial algorithm's
semantics) Example 1 needs no remedy, Examples 2, 3 and 5 do."""

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
eik = pytest.importorskip("paper_2106_15869_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SCHEDULE = {"node": dict(variant="node"), "tile": dict(variant="tile"), "fim": dict(variant="fim"),
            "fifo": dict(variant="tile", fifo=True)}


@pytest.mark.parametrize("variant", list(SCHEDULE))
@pytest.mark.parametrize("n", [200, 500])
@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_examples_match_oracle(k, n, variant):
    P = W.paper_example(k, n)
    print(f"[case] {P.name} {variant}", flush=True)
    got = eik.solve(torch.from_numpy(P.F).to(DEV), P.h, P.sources, source_values=P.source_values,
                    **SCHEDULE[variant]).cpu().numpy()
    ref = oracle.fmm(P.F.astype(np.float64), P.h, P.sources, values=P.source_values)
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got - ref)) <= 1e-5 * ref.max()


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_update_step_claims(k):
    P = W.paper_example(k, 200, dtype=np.float64)
    F = torch.from_numpy(P.F).to(DEV)
    ref = oracle.fmm(P.F, P.h, P.sources, values=P.source_values)
    upd = eik.solve(F, P.h, P.sources, source_values=P.source_values, variant="node", deterministic=True,
                    skip_remedy=True).cpu().numpy()
    full, st = eik.solve(F, P.h, P.sources, source_values=P.source_values, variant="node", deterministic=True,
                         stats=True)
    assert np.array_equal(full.cpu().numpy(), ref)
    if k == 1:
        assert np.array_equal(upd, ref) and st["remedy_initial"] == 0
    else:
        assert np.any(upd > ref * (1 + 1e-12)) and st["remedy_initial"] > 0


_FULL_REF = {}  # the oracle's solution of the last full-size example (shared by its schedules)


def _full_ref(P, key):
    if key not in _FULL_REF:
        _FULL_REF.clear()
        _FULL_REF[key] = oracle.fmm(P.F.astype(np.float64), P.h, P.sources, values=P.source_values)
    return _FULL_REF[key]


@pytest.mark.parametrize("variant", ["tile", "fim"])
@pytest.mark.parametrize("n", [2000, 4000])
@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_examples_full_size_float32(k, n, variant):
    """The paper's largest grids (2000^2 and 4000^2) in float32, default tile
    schedule and FIM, against the float64 oracle on every node.  At these
    sizes the float32 fixed point itself can lie farther than 1e-5 max phi
    from the float64 one: storing phi ~ 10 with steps of h = 0.005 rounds
    every step of a front the same way within a binade (Example 1 at 4000^2:
    1.45e-5 max phi, the same with the local root formed in float64; the
    oracle's own float32 emulation of Algorithm 2 drifts 1.7e-6 at 1000^2 and
    5.8e-6 at 2000^2).  So the gates are: every value finite, every node a
    float32 fixed point (<= 4 ulp, float64 G on the output), and the error
    within the causal-chain bound derived from that residual (chain_bound);
    the 1e-5 max phi figure is reported.  The float64 mode below meets the
    1e-12 max phi gate at the same sizes."""
    from tests.oracle_checks import chain_bound, fixed_point_ulps
    P = W.paper_example(k, n)
    print(f"[case] {P.name} {variant} float32", flush=True)
    got = eik.solve(torch.from_numpy(P.F).to(DEV), P.h, P.sources, source_values=P.source_values,
                    **SCHEDULE[variant]).cpu().numpy()
    ref = _full_ref(P, (k, n, "f32"))
    assert np.all(np.isfinite(got))
    err = float(np.max(np.abs(got - ref)))
    ulps = fixed_point_ulps(P.F, P.h, got, P.sources)
    bound = chain_bound(P.F, P.h, P.sources, got, P.source_values)
    print(f"[err] {err / ref.max():.3e} of max phi (1e-5 gate: {'met' if err <= 1e-5 * ref.max() else 'not met'}), "
          f"fixed point {ulps.max():.2f} ulp, chain bound {bound / ref.max():.3e} of max phi", flush=True)
    assert ulps.max() <= 4.0
    assert err <= bound


@pytest.mark.parametrize("n", [2000, 4000])
@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_examples_full_size_float64(k, n):
    """The same grids in the float64 mode (tile schedule): within 1e-12 max phi
    of the oracle on every node."""
    P = W.paper_example(k, n, dtype=np.float64)
    print(f"[case] {P.name} tile float64", flush=True)
    got = eik.solve(torch.from_numpy(P.F).to(DEV), P.h, P.sources, source_values=P.source_values).cpu().numpy()
    ref = _full_ref(P, (k, n, "f64"))
    err = float(np.max(np.abs(got - ref)))
    print(f"[err] {err / ref.max():.3e} of max phi", flush=True)
    assert np.all(np.isfinite(got))
    assert err <= 1e-12 * ref.max()
