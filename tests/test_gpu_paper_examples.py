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
