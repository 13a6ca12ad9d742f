"""GPU parity with per-axis grid spacing (Eq 5 with dx != dy, Algorithm 1.2,
and its 3D analogue) against the oracle's anisotropic solvers: the dense
local solve bit for bit, full solves of every schedule within the float32 /
float64 gates, and the adjoint on the GPU's own solution."""

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
eik = pytest.importorskip("paper_2106_15869_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {np.float32: 1e-5, np.float64: 1e-12}
SCHEDULE = {"node": dict(variant="node"), "tile": dict(variant="tile"), "fim": dict(variant="fim"),
            "fifo": dict(variant="tile", fifo=True)}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape,sp", [((37, 53), (0.4, 1.7)), ((9, 13, 17), (2.0, 0.5, 1.1))])
def test_apply_local_bitwise(shape, sp, dtype):
    r = np.random.default_rng(len(shape))
    F = np.exp(r.uniform(-2, 2, size=shape))
    F[r.random(shape) < 0.1] = 0.0
    phi = r.uniform(0, 5, size=shape)
    phi[r.random(shape) < 0.2] = np.inf
    F, phi = F.astype(dtype), phi.astype(dtype)
    got = eik.apply_local(dev(F), dev(phi), None, spacing=sp).cpu().numpy()
    want = oracle.apply_local(F, 1.0, phi, dtype=dtype, spacing=sp)
    assert np.array_equal(got, want)


def _cases():
    r = np.random.default_rng(31)
    out = []
    for k, (shape, sp) in enumerate([((64, 90), (0.3, 1.2)), ((120, 41), (2.0, 0.7)), ((1, 60), (5.0, 0.25)),
                                     ((20, 24, 18), (0.5, 1.0, 2.0)), ((33, 9, 40), (1.3, 0.4, 0.9))]):
        F = np.exp(r.uniform(-1, 1, size=shape))
        if k % 2:
            F[r.random(shape) < 0.08] = 0.0
        src = r.choice(F.size, size=2, replace=False)
        out.append((f"aniso_{k}", F, sp, src))
    P = W.maze_3d(32)
    out.append(("maze32", P.F.astype(np.float64), (0.5, 1.0, 2.0), P.sources))
    return out


@pytest.mark.parametrize("variant", ["node", "tile", "fim", "fifo"])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_solve_matches_oracle(case, dtype, variant):
    name, F, sp, src = case
    print(f"[case] aniso {name} {np.dtype(dtype).name} {variant}", flush=True)
    Fd = F.astype(dtype)
    got = eik.solve(dev(Fd), None, src, spacing=sp, **SCHEDULE[variant]).cpu().numpy()
    ref = oracle.fmm(Fd.astype(np.float64), 1.0, src, spacing=sp)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(got))
    err = np.max(np.abs(got[fin].astype(np.float64) - ref[fin]))
    assert err <= TOL[dtype] * ref[fin].max(), err


@pytest.mark.parametrize("case", _cases()[:4], ids=lambda c: c[0])
def test_adjoint_matches_oracle(case):
    name, F, sp, src = case
    r = np.random.default_rng(5)
    g = np.where(r.random(F.shape) < 0.05, r.uniform(0.5, 2.0, F.shape), 0.0)
    Fd = dev(F.astype(np.float64))
    phi = eik.solve(Fd, None, src, spacing=sp)
    d = eik.adjoint(Fd, phi, None, src, dev(g), spacing=sp).cpu().numpy()
    want = oracle.adjoint(F, 1.0, src, phi.cpu().numpy(), g, spacing=sp)
    assert np.max(np.abs(d - want)) <= 1e-9 * max(np.max(np.abs(want)), 1e-300)


def test_equal_spacing_matches_isotropic():
    P = W.lognormal_2d(128, seed=9)
    F = dev(P.F.astype(np.float64))
    a = eik.solve(F, P.h, P.sources).cpu().numpy()
    b = eik.solve(F, None, P.sources, spacing=(P.h, P.h)).cpu().numpy()
    assert np.max(np.abs(a - b)) <= 1e-13 * a.max()


@pytest.mark.parametrize("case", [_cases()[0], _cases()[3]], ids=lambda c: c[0])
def test_tune_with_spacing(case):
    """eik_tune with per-axis spacing times only the shapes that support it,
    its choice solves within the float32 gate, and the isotropic problem of
    the same size class is tuned on its own (separate cache entry)."""
    name, F, sp, src = case
    print(f"[case] tune aniso {name}", flush=True)
    Fd = dev(F.astype(np.float32))
    t = eik.tune(Fd, None, src, spacing=sp)
    default = (1, 16, 16) if F.ndim == 2 else (8, 8, 8)
    assert t["candidates"], "first call for this class times candidates"
    got = eik.solve(Fd, None, src, spacing=sp, tile=t["tile"], inner_iters=t["inner_iters"]).cpu().numpy()
    ref = oracle.fmm(F.astype(np.float32).astype(np.float64), 1.0, src, spacing=sp)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(got))
    assert np.max(np.abs(got[fin] - ref[fin])) <= TOL[np.float32] * ref[fin].max()
    # the isotropic problem of the same size class has its own cache entry
    # (tuned here for the first-in first-out remedy, a class no other test
    # tunes, so that the timing is not served from an earlier test's entry)
    iso = eik.tune(Fd, 1.0, src, fifo=True)
    assert iso["candidates"] and any(c["tile"] not in {(0, 0, 0), default} for c in iso["candidates"])
    # with spacing the zero tile (the same configuration as the default
    # shapes then) is not timed twice
    assert all(c["tile"] == default for c in t["candidates"])
