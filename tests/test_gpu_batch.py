"""GPU parity of the batched entry points (eik_solve_batch / eik_adjoint_batch)
and of graph-captured solves.

Each grid of a batch is compared with the oracle's fast marching solution of
that grid alone (float32: 1e-5 x max phi, float64: 1e-12 x max phi, identical
+inf masks), and the batched adjoint with the oracle's reverse sweep.  Grids of
mixed shapes, spacings, source counts and source values, ragged against the
tile size, including 1-wide strips and a single node."""

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
eik = pytest.importorskip("paper_2106_15869_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {np.float32: 1e-5, np.float64: 1e-12}


def _grids(nd, seed, count):
    r = np.random.default_rng(seed)
    out = []
    for k in range(count):
        if nd == 2:
            sh = (int(r.integers(1, 90)), int(r.integers(1, 130)))
        else:
            sh = tuple(int(v) for v in r.integers(1, 22, size=3))
        F = np.exp(r.uniform(-1.5, 1.5, size=sh))
        if k % 3 == 1:
            F[r.random(sh) < 0.1] = 0.0
        n = int(np.prod(sh))
        src = r.choice(n, size=min(n, int(r.integers(1, 5))), replace=False)
        vals = r.uniform(0, 2, size=len(src)) if k % 4 == 2 else np.zeros(len(src))
        out.append((F, float(r.uniform(0.2, 2.0)), src, vals))
    out.append((np.ones((1, 1)) if nd == 2 else np.ones((1, 1, 1)), 1.0, np.array([0]), np.zeros(1)))
    return out


def _pack(grids, dtype):
    F = np.concatenate([g[0].astype(dtype).ravel() for g in grids])
    return torch.from_numpy(F).to(DEV)


def _check_grid(got, F, h, src, vals, dtype):
    ref = oracle.fmm(F.astype(dtype).astype(np.float64), h, src, values=vals)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(got))
    if fin.any():
        err = np.max(np.abs(got[fin].astype(np.float64) - ref[fin]))
        assert err <= TOL[dtype] * np.max(np.abs(ref[fin])) + 1e-300, err
    return ref


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("nd,seed", [(2, 1), (2, 2), (3, 3)])
def test_batch_matches_oracle_per_grid(nd, seed, dtype):
    grids = _grids(nd, seed, 14 if nd == 2 else 8)
    shapes = [g[0].shape for g in grids]
    print(f"[case] batch nd={nd} seed={seed} {np.dtype(dtype).name} shapes={shapes}", flush=True)
    F = _pack(grids, dtype)
    phi, st = eik.solve_batch(F, shapes, [g[1] for g in grids], [g[2] for g in grids],
                              source_values=[g[3] for g in grids], stats=True)
    torch.cuda.synchronize()
    for (Fg, h, src, vals), p in zip(grids, eik.unpack(phi, shapes)):
        _check_grid(p.cpu().numpy(), Fg, h, src, vals, dtype)
    assert st["evals_detect"] == F.numel() - sum(len(np.unique(g[2])) for g in grids)


def test_batch_of_workloads_and_single_solves_agree():
    """Grids of the benchmark recipes batched together give what each gives
    solved alone (both within the float32 gate of the oracle)."""
    Ps = [W.lognormal_2d(200, seed=1), W.lognormal_2d(96, seed=2),
          W.Problem("maze2d", W.maze_field((150, 180), 4, free_coord=(0, 0)), 1.0, np.array([0])),
          W.lognormal_2d(33, seed=3)]
    shapes = [P.F.shape for P in Ps]
    F = eik.pack([torch.from_numpy(P.F).to(DEV) for P in Ps])
    phi = eik.solve_batch(F, shapes, [P.h for P in Ps], [P.sources for P in Ps])
    for P, p in zip(Ps, eik.unpack(phi, shapes)):
        alone = eik.solve(torch.from_numpy(P.F).to(DEV), P.h, P.sources).cpu().numpy()
        ref = _check_grid(p.cpu().numpy(), P.F, P.h, P.sources, None, np.float32)
        assert np.max(np.abs(alone - p.cpu().numpy())) <= 2e-5 * ref.max()


@pytest.mark.parametrize("nd", [2, 3])
def test_adjoint_batch_matches_oracle(nd):
    grids = _grids(nd, 10 + nd, 6)
    shapes = [g[0].shape for g in grids]
    print(f"[case] adjoint batch nd={nd} shapes={shapes}", flush=True)
    F = _pack(grids, np.float64)
    hs = [g[1] for g in grids]
    srcs = [g[2] for g in grids]
    r = np.random.default_rng(nd)
    gs = [np.where(r.random(g[0].shape) < 0.05, r.uniform(0.5, 2.0, g[0].shape), 0.0) for g in grids]
    phi = eik.solve_batch(F, shapes, hs, srcs)
    G = torch.from_numpy(np.concatenate([g.ravel() for g in gs])).to(DEV)
    d = eik.adjoint_batch(F, phi, shapes, hs, srcs, G)
    for (Fg, h, src, vals), gk, dk, pk in zip(grids, gs, eik.unpack(d, shapes), eik.unpack(phi, shapes)):
        ph = pk.cpu().numpy()
        _check_grid(ph, Fg, h, src, None, np.float64)
        # the oracle's reverse sweep on the GPU's solution: same upwind stencils
        want = oracle.adjoint(Fg, h, src, ph, gk)
        got = dk.cpu().numpy()
        assert np.max(np.abs(got - want)) <= 1e-9 * max(np.max(np.abs(want)), 1e-300)


@pytest.mark.parametrize("variant", ["tile", "node"])
def test_graph_capture_replays(variant):
    """A solve enqueued with async_=True captured in a graph: every replay,
    with eager work in between, gives the oracle's solution."""
    P = W.lognormal_2d(160, seed=7)
    F = torch.from_numpy(P.F.astype(np.float64)).to(DEV)
    out = torch.empty_like(F)
    ws = torch.empty(eik.eik_workspace_size(P.F.shape, eik.make_options(eik.EIK_FLOAT64, variant)),
                     dtype=torch.uint8, device=DEV)
    cap = 2000 if variant == "node" else 300
    # the eager async run also warms up the stream for capture
    eik.solve(F, P.h, P.sources, variant=variant, out=out, workspace=ws, max_iters=cap, async_=True)
    torch.cuda.synchronize()
    ref = oracle.fmm(P.F.astype(np.float64), P.h, P.sources)
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= 1e-12 * ref.max()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            eik.solve(F, P.h, P.sources, variant=variant, out=out, workspace=ws, max_iters=cap, async_=True,
                      stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        out.fill_(-1.0)
        junk = torch.randn(1 << 16, device=DEV).sum()  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 1e-12 * ref.max(), (rep, float(junk))


def test_graph_capture_replays_3d_with_early_remedy():
    """3D float32 solve (early remedy visits in the update step) enqueued with
    async_=True and captured in a graph: every replay, with eager work in
    between, meets the float32 gate and reports that its loops emptied."""
    P = W.maze_3d(40, seed=3)
    F = torch.from_numpy(P.F).to(DEV)
    out = torch.empty_like(F)
    ws = torch.empty(eik.eik_workspace_size(P.F.shape, eik.make_options(eik.EIK_FLOAT32, "tile")),
                     dtype=torch.uint8, device=DEV)
    _, st = eik.solve(F, P.h, P.sources, stats=True)
    assert st["evals_early"] > 0
    cap = int(1.25 * max(st["step2_iters"], st["step3_iters"])) + 32
    ref = oracle.fmm(P.F.astype(np.float64), P.h, P.sources)
    eik.solve(F, P.h, P.sources, out=out, workspace=ws, max_iters=cap, async_=True)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            eik.solve(F, P.h, P.sources, out=out, workspace=ws, max_iters=cap, async_=True, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        out.fill_(-1.0)
        junk = torch.randn(1 << 16, device=DEV).sum()  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        eik.check_async(ws)
        got = out.cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 1e-5 * ref.max(), (rep, float(junk))


@pytest.mark.parametrize("P", [W.lognormal_2d(300, seed=4), W.maze_3d(48)], ids=lambda P: P.name)
def test_tune_picks_a_candidate_and_caches_it(P):
    """eik_tune times the shapes, then the ordered remedy's per-launch minimum
    (half and twice the default) and the workgroups per launch for the chosen
    shape; it returns the fastest candidate, caches it, and the choice solves
    within the float32 gate."""
    F = torch.from_numpy(P.F).to(DEV)
    t = eik.tune(F, P.h, P.sources)
    cands = t["candidates"]
    assert cands, "first call for this size class times candidates"

    def key(c):
        return (c["tile"], c["inner_iters"], c["order_min"], c["workgroups"])

    assert key(t) in {key(c) for c in cands}
    assert min(c["ms"] for c in cands) == pytest.approx([c["ms"] for c in cands if key(c) == key(t)][0])
    default_om = 512 if P.F.ndim == 2 else 1024
    assert {c["order_min"] for c in cands} == {0, default_om // 2, 2 * default_om}
    assert {c["workgroups"] for c in cands} == ({0, 1024, 2048} if P.F.ndim == 3 else {0, 1024, 1536})
    again = eik.tune(F, P.h, P.sources)
    assert again["candidates"] == [] and key(again) == key(t)
    phi = eik.solve(F, P.h, P.sources, tile=t["tile"], inner_iters=t["inner_iters"], order_min=t["order_min"],
                    workgroups=t["workgroups"]).cpu().numpy()
    ref = oracle.fmm(P.F.astype(np.float64), P.h, P.sources)
    assert np.max(np.abs(phi - ref)) <= 1e-5 * ref.max()


@pytest.mark.parametrize("order_min,workgroups", [(1, 8), (64, 1024), (4096, 2048), (0, 8)])
@pytest.mark.parametrize("P", [W.lognormal_2d(200, seed=6), W.maze_3d(48), W.layered_3d(40)],
                         ids=lambda P: P.name)
def test_schedule_options_keep_the_fixed_point(P, order_min, workgroups):
    """Explicit per-launch minimum of the ordered remedy and persistent
    workgroups per launch (down to 8, one per sub-list) change only the order
    of the tile visits: the result meets the float32 gate, for a single grid
    and for a batch of two."""
    print(f"[case] {P.name} order_min {order_min} workgroups {workgroups}", flush=True)
    F = torch.from_numpy(P.F).to(DEV)
    ref = oracle.fmm(P.F.astype(np.float64), P.h, P.sources)
    fin = np.isfinite(ref)
    phi = eik.solve(F, P.h, P.sources, order_min=order_min, workgroups=workgroups).cpu().numpy()
    assert np.array_equal(fin, np.isfinite(phi))
    assert np.max(np.abs(phi[fin] - ref[fin])) <= 1e-5 * ref[fin].max()
    Fb = torch.cat([F.reshape(-1), F.reshape(-1)])
    pb = eik.solve_batch(Fb, [P.F.shape] * 2, P.h, [P.sources] * 2, order_min=order_min,
                         workgroups=workgroups).cpu().numpy()
    for k in range(2):
        part = pb[k * P.F.size:(k + 1) * P.F.size].reshape(P.F.shape)
        assert np.array_equal(fin, np.isfinite(part))
        assert np.max(np.abs(part[fin] - ref[fin])) <= 1e-5 * ref[fin].max()
