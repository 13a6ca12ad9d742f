#!/usr/bin/env python3
"""Benchmark: IFIM eikonal solve, 3D 256^3 float32 maze, one MI355X.

Workload: grid 256^3, h = 1; blocks of 8^3 cells are obstacles (F = 0.001)
with probability 0.3, else free (F = 1); source (0,0,0), its block forced
free.  One step = one complete forward solve (initialisation, update step,
remedy step) with the default (tile) schedule.  Inputs are resident in HBM and
the workspace is preallocated before the timed region; value = grid nodes
solved per second.

Also reported: forward + adjoint (dL/dF for L = sum of phi at 64 receivers on
the far face z = 255), the plain node-list schedule, the tile schedule with a
first-in first-out remedy, the fast iterative method (FIM, the paper's
baseline) on the same node lists, the dominant kernel's achieved bandwidth
against the 8 TB/s HBM peak (device time from HIP events on the library's
stream; bytes = 8 per local-solver evaluation + 4 per changed value, from the
solve's own counters), the whole solve against the 28 B/node floor, and the
float64 fast-marching oracle on the host as a CPU baseline (median of 3 runs).

Other modes: --configs (a table of the five workload configurations, GPU
beside the oracle), --replay (the paper's Examples 1, 2, 3, 5), --batch N
(N uneven 2D grids, forward + adjoint in one captured graph).

Prints ONE JSON line.  --gpus N with N > 1 exits: this build runs on one GPU.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variant", default="tile", choices=["tile", "node"])
    ap.add_argument("--n", type=int, default=256, help="grid side of the 3D maze")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip adjoint and node-list timings")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run one device-to-device copy of MIB MiB (for scaling HBM counters)")
    ap.add_argument("--replay", action="store_true",
                    help="instead: the paper's Examples 1, 2, 3, 5 at 200^2 .. 4000^2 with every schedule")
    ap.add_argument("--batch", type=int, default=0, metavar="COUNT",
                    help="instead: COUNT uneven 2D lognormal grids (sides 128..2048) solved forward + adjoint "
                         "in one captured graph with a tuned tile")
    ap.add_argument("--configs", action="store_true",
                    help="instead: the five workload configurations, GPU time beside the oracle's")
    return ap.parse_args()


# The paper's own timings (seconds; Tables 1, 2, 3, 5; improved method and FIM
# on its GPU), quoted as context for the replay, not as a target.
PAPER_SECONDS = {
    1: {"ifim": (0.00141, 0.00384, 0.03721, 0.11642, 0.80981), "fim": (0.00164, 0.00428, 0.08834, 0.32604, 1.67655)},
    2: {"ifim": (0.00097, 0.00329, 0.0539, 0.35359, 1.09434), "fim": (0.00118, 0.00319, 0.08794, 0.63421, 1.86989)},
    3: {"ifim": (0.00089, 0.00341, 0.0499, 0.36897, 1.48971), "fim": (0.00125, 0.00410, 0.08954, 0.78251, 2.05581)},
    5: {"ifim": (0.00119, 0.00341, 0.0689, 0.56897, 1.098971), "fim": (0.00125, 0.00410, 0.08954, 0.78251, 2.45581)},
}


def batch_bench(torch, eik, W, count, steps):
    """Many independent 2D grids (the batch recipe): tile shape from eik_tune on
    the largest grid; one eager forward + adjoint (stats, loop lengths); then
    forward + adjoint enqueued asynchronously with a fixed launch budget,
    captured in one graph and replayed; parity of a seeded sample of 8 grids
    against the float64 oracle."""
    import oracle
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    Ps = W.batch_2d(count)
    gen_s = time.perf_counter() - t0
    print(f"[batch] generated {count} grids in {gen_s:.1f} s", file=sys.stderr, flush=True)
    shapes = [P.F.shape for P in Ps]
    hs = [P.h for P in Ps]
    srcs = [P.sources for P in Ps]
    F = torch.from_numpy(np.concatenate([P.F.ravel() for P in Ps])).to(dev)
    g = np.concatenate([np.where(np.isin(np.arange(P.F.size), P.receivers), 1.0, 0.0) for P in Ps])
    G = torch.from_numpy(g.astype(np.float32)).to(dev)
    n = F.numel()
    big = max(Ps, key=lambda P: P.F.size)
    tuned = eik.tune(torch.from_numpy(big.F).to(dev), big.h, big.sources)
    kw = dict(tile=tuned["tile"], inner_iters=tuned["inner_iters"])
    print(f"[batch] tuned: {kw}", file=sys.stderr, flush=True)
    phi, st = eik.solve_batch(F, shapes, hs, srcs, stats=True, **kw)
    d, sta = eik.adjoint_batch(F, phi, shapes, hs, srcs, G, stats=True)
    torch.cuda.synchronize()
    # eager timing
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        eik.solve_batch(F, shapes, hs, srcs, out=phi, **kw)
        eik.adjoint_batch(F, phi, shapes, hs, srcs, G, out=d)
    e1.record()
    torch.cuda.synchronize()
    eager_ms = e0.elapsed_time(e1) / steps
    # fixed launch budgets from the eager run, then one captured graph
    budget = int(1.25 * max(st["step2_iters"], st["step3_iters"])) + 32
    abudget = int(1.25 * sta["step3_iters"]) + 32
    opt = eik.make_options(eik.EIK_FLOAT32, "tile", tile=kw["tile"])
    ws = torch.empty(eik.eik_batch_workspace_size(shapes, hs, srcs, opt), dtype=torch.uint8, device=dev)
    wa = torch.empty(eik.eik_adjoint_batch_workspace_size(shapes, hs, srcs, opt), dtype=torch.uint8, device=dev)
    phi_g, d_g = torch.empty_like(F), torch.empty_like(F)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())

    def enqueue():
        eik.solve_batch(F, shapes, hs, srcs, out=phi_g, workspace=ws, max_iters=budget, async_=True, stream=s, **kw)
        eik.adjoint_batch(F, phi_g, shapes, hs, srcs, G, out=d_g, workspace=wa, max_iters=abudget, async_=True,
                          stream=s)
    with torch.cuda.stream(s):
        enqueue()  # warm-up of the async path on the capture stream
    s.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            enqueue()
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1) / steps
    # every loop of the last replay emptied its lists within its budget
    eik.check_async(ws)
    eik.check_async(wa)
    print(f"[batch] eager {eager_ms:.1f} ms, graph {graph_ms:.1f} ms", file=sys.stderr, flush=True)
    # parity on a sample
    r = np.random.default_rng(W.BASE_SEED)
    sample = sorted(int(i) for i in r.choice(len(Ps), size=min(8, len(Ps)), replace=False))
    offs = np.concatenate([[0], np.cumsum([P.F.size for P in Ps])])
    phis, ds = phi_g.cpu().numpy(), d_g.cpu().numpy()
    worst_phi, worst_adj = 0.0, 0.0
    for i in sample:
        P = Ps[i]
        got = phis[offs[i]:offs[i + 1]].reshape(P.F.shape).astype(np.float64)
        ref = oracle.fmm(P.F.astype(np.float64), P.h, P.sources)
        worst_phi = max(worst_phi, float(np.max(np.abs(got - ref)) / ref.max()))
        gi = g[offs[i]:offs[i + 1]].reshape(P.F.shape)
        dref = oracle.adjoint(P.F.astype(np.float64), P.h, P.sources, got, gi)
        dg = ds[offs[i]:offs[i + 1]].reshape(P.F.shape)
        worst_adj = max(worst_adj, float(np.max(np.abs(dg - dref)) / np.max(np.abs(dref))))
    return {"metric": "batched forward + adjoint, node-updates/s", "value": n / (graph_ms / 1e3),
            "unit": "node-updates/s", "n_gpus": 1, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{count} 2D lognormal grids, sides U{{128..2048}}, 1-8 sources each, "
                                   "16 receivers on the last row (L = sum of phi there)", "nodes": n,
                       "tile": list(kw["tile"]), "inner_iters": kw["inner_iters"]},
            "graph_ms_per_step": graph_ms, "eager_ms_per_step": eager_ms,
            "launch_budget": {"forward": budget, "adjoint": abudget}, "async_status": "EIK_OK",
            "tune": tuned, "stats_forward": st, "stats_adjoint": sta,
            "parity_sample": {"instances": sample, "max_err_rel_phi": worst_phi,
                              "adjoint_max_err_rel": worst_adj},
            "host_generation_s": gen_s}


def replay(torch, eik, W):
    """Examples 1, 2, 3, 5 of the paper at its grid sizes: solve ms per
    schedule (median of 3 after a warm-up, HIP events), evaluation counts, and
    the float32 gate against the float64 oracle up to 1000^2."""
    import oracle
    dev = torch.device("cuda:0")
    rows = []
    schedules = {"tile": dict(variant="tile"), "node": dict(variant="node"), "fim": dict(variant="fim")}
    for k in (1, 2, 3, 5):
        for j, n in enumerate(W.PAPER_SIZES):
            P = W.paper_example(k, n)
            F = torch.from_numpy(P.F).to(dev)
            phi = torch.empty_like(F)
            ref = oracle.fmm(P.F.astype(np.float64), P.h, P.sources, values=P.source_values) if n <= 1000 else None
            row = {"example": k, "n": n, "sources": int(len(P.sources)),
                   "paper_s": {m: PAPER_SECONDS[k][m][j] for m in ("ifim", "fim")}}
            for name, kw in schedules.items():
                def run():
                    return eik.solve(F, P.h, P.sources, source_values=P.source_values, out=phi, **kw)
                _, st = eik.solve(F, P.h, P.sources, source_values=P.source_values, out=phi, stats=True, **kw)
                times = []
                for _ in range(3):
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record()
                    run()
                    e1.record()
                    torch.cuda.synchronize()
                    times.append(e0.elapsed_time(e1))
                entry = {"ms": sorted(times)[1],
                         "evals": st["evals_step2"] + st["evals_detect"] + st["evals_remedy"] + st["evals_check"]
                         + st["evals_early"]}
                if ref is not None:
                    entry["max_err_rel"] = float(np.max(np.abs(phi.cpu().numpy() - ref)) / ref.max())
                row[name] = entry
            rows.append(row)
            print(json.dumps({"progress": f"example {k} n {n}", **{m: row[m]["ms"] for m in schedules}}),
                  file=sys.stderr, flush=True)
    return rows


def alg_bytes(kind, st, esz=4):
    """Bytes the method must move for one kernel kind over a whole solve, in
    the unit of the scope table: one local-solver evaluation reads the node's
    F and phi (2 * esz; neighbour values come from the same staged tile), and
    every value that changes is written once (esz).  Detection evaluates
    every non-source node and writes nothing.  The update kernel also runs
    the early remedy visits (3D): their evaluations count there (their
    writes are not counted)."""
    if kind == "update":
        return 2 * esz * (st["evals_step2"] + st["evals_early"]) + esz * st["written_step2"]
    if kind == "remedy":
        return 2 * esz * st["evals_remedy"] + esz * st["written_step3"]
    if kind == "detect":
        return 2 * esz * st["evals_detect"]
    return None


def staged_bytes(kind, st, variant, n_nodes, tile_nodes, esz=4):
    """Bytes a kernel kind stages over a whole solve (second view): a tile
    visit reads every node's F and phi (2 * esz) and label (1 B) into LDS and
    writes back the changed values (esz, plus the label in the update step);
    a node-list evaluation adds about 9 B of list and label traffic."""
    if kind == "detect":
        return n_nodes * (2 * esz + 1)
    if variant == "tile":
        if kind == "update":
            return st["tile_visits_step2"] * tile_nodes * (2 * esz + 1) + st["written_step2"] * (esz + 1)
        if kind == "remedy":
            return st["tile_visits_step3"] * tile_nodes * (2 * esz + 1) + st["written_step3"] * esz
    else:
        if kind == "update":
            return st["evals_step2"] * (2 * esz + 9) + st["written_step2"] * esz
        if kind == "remedy":
            return st["evals_remedy"] * (2 * esz + 9) + st["written_step3"] * esz
    return None


def _elf_sections(data):
    """Section headers of a little-endian ELF64 image: {name: header tuple}."""
    import struct
    shoff = struct.unpack_from("<Q", data, 0x28)[0]
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", data, 0x3A)
    raw = [struct.unpack_from("<IIQQQQIIQQ", data, shoff + i * shentsize) for i in range(shnum)]
    stroff = raw[shstrndx][4]
    named = {data[stroff + h[0]:data.index(b"\0", stroff + h[0])].decode(): h for h in raw}
    return named, raw


def kernel_code_hash(symbol_part, lib_path=None):
    """SHA-256 (16 hex digits) of the gfx950 machine code of every kernel whose
    symbol contains `symbol_part`, read from the built library's offload
    bundles: it changes exactly when that kernel's code does."""
    import hashlib
    import re
    import struct
    lib_path = lib_path or os.path.join(ROOT, "paper_2106_15869_amd", "libeik.so")
    data = open(lib_path, "rb").read()
    fb = _elf_sections(data)[0][".hip_fatbin"]
    sec = data[fb[4]:fb[4] + fb[5]]
    found = []
    for m in re.finditer(b"__CLANG_OFFLOAD_BUNDLE__", sec):
        b = m.start()
        p = b + 32
        for _ in range(struct.unpack_from("<Q", sec, b + 24)[0]):
            off, size, tl = struct.unpack_from("<QQQ", sec, p)
            triple = sec[p + 24:p + 24 + tl].decode()
            p += 24 + tl
            if "gfx950" not in triple:
                continue
            co = sec[b + off:b + off + size]
            named, raw = _elf_sections(co)
            text, symtab = named[".text"], named[".symtab"]
            strtab = raw[symtab[6]]
            for k in range(symtab[5] // 24):
                nm, info, _, _, val, sz = struct.unpack_from("<IBBHQQ", co, symtab[4] + 24 * k)
                name = co[strtab[4] + nm:co.index(b"\0", strtab[4] + nm)].decode()
                if (info & 0xF) == 2 and sz and symbol_part in name:
                    o = text[4] + val - text[3]
                    found.append((name, co[o:o + sz]))
    if not found:
        return None
    h = hashlib.sha256()
    for _, code in sorted(found):
        h.update(code)
    return h.hexdigest()[:16]


def measured_traffic(kernel, code_hash):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 --pmc
    summary, if it was taken on the kernel's current machine code (its
    record carries kernel_code_hash of the profiled build); else None."""
    import glob
    if code_hash is None:
        return None
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if not line.startswith("traffic_json:"):
                continue
            rec = json.loads(line.split(":", 1)[1])
            if rec.get("kernel") == kernel and rec.get("code_sha16") == code_hash:
                return rec["bytes_per_launch"]
    return None


def host_cpu():
    """CPU model (lscpu) and the logical CPUs this process may run on."""
    import subprocess
    model = None
    try:
        for line in subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:  # noqa: BLE001 -- the record only
        pass
    if model is None and os.path.exists("/proc/cpuinfo"):
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def oracle_time(fn, max_runs=3, single_if_over_s=10.0):
    """Median wall time (s) of `fn` over up to three runs; one run when the
    first takes longer than single_if_over_s."""
    times = []
    for _ in range(max_runs):
        t0 = time.perf_counter()
        fn()
        times.append(time.perf_counter() - t0)
        if times[0] > single_if_over_s:
            break
    return float(np.median(times)), times


def timed(torch, fn, steps, warmup, stream):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, (time.perf_counter() - t0) * 1e3 / steps


def cpu_baseline(P):
    """The float64 fast-marching oracle on the same workload, single thread,
    median of 3 runs (one run if it takes over 10 s)."""
    import oracle
    F64 = P.F.astype(np.float64)
    med, runs = oracle_time(lambda: oracle.fmm(F64, P.h, P.sources))
    return {"value": P.n / med, "unit": "node-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"full {P.name} solves ({P.n} nodes) by the float64 heap-ordered fast-marching "
                      f"oracle, single thread, median of {len(runs)}: "
                      + ", ".join(f"{t:.2f}" for t in runs) + " s",
            "host": host_cpu()}


def _gpu_ms(torch, fn, steps, warmup=1):
    """Median device time (ms) of fn over `steps` runs (HIP events on the
    current stream) after `warmup` runs."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times))


def configs_table(torch, eik, W, steps):
    """The five workload configurations: GPU ms per schedule (median, HIP
    events, inputs resident) beside the float64 oracle on the host (median of
    3 single-thread runs, or one over 10 s; the batch on a thread pool over
    every usable host CPU) and the float32-vs-oracle error."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    dev = torch.device("cuda:0")
    rows = []

    def row(name, P, schedules, fwd_adjoint=None):
        F = torch.from_numpy(P.F).to(dev)
        phi = torch.empty_like(F)
        F64 = P.F.astype(np.float64)
        ref = oracle.fmm(F64, P.h, P.sources)
        fin = np.isfinite(ref)
        r = {"config": name, "nodes": P.n, "dtype": str(P.F.dtype)}
        for sname, kw in schedules.items():
            run = lambda: eik.solve(F, P.h, P.sources, P.eps, out=phi, **kw)  # noqa: E731
            ms = _gpu_ms(torch, run, steps)
            got = phi.cpu().numpy().astype(np.float64)
            err = float(np.max(np.abs(got[fin] - ref[fin])) / ref[fin].max())
            r[sname] = {"ms": ms, "node_updates_per_s": P.n / (ms / 1e3), "max_err_rel": err}
        med, runs = oracle_time(lambda: oracle.fmm(F64, P.h, P.sources))
        r["oracle"] = {"ms": med * 1e3, "runs_s": runs, "node_updates_per_s": P.n / med, "cores": 1}
        if fwd_adjoint is not None:
            r.update(fwd_adjoint(F, ref))
        rows.append(r)
        print(json.dumps({"progress": name, **{k: v for k, v in r.items() if isinstance(v, dict)}}),
              file=sys.stderr, flush=True)

    row("1: 64^2 FP64, F = 1, source (32,32), eps 1e-12", W.tiny_constant(),
        {"node": dict(variant="node"), "tile": dict(variant="tile")})
    row("2: 4096^2 FP32 lognormal, source (0,0)", W.lognormal_2d(4096),
        {"node": dict(variant="node"), "tile": dict(variant="tile")})
    row("3: 256^3 FP32 maze, source (0,0,0)", W.maze_3d(256),
        {"node": dict(variant="node"), "tile": dict(variant="tile")})

    P4 = W.layered_3d(192)

    def misfit(F, ref):
        """Forward + adjoint of L = sum_r (phi_r - t_obs,r)^2, t_obs = phi(F_obs)."""
        rec = torch.from_numpy(P4.receivers).to(dev)
        t_obs = eik.solve(torch.from_numpy(P4.meta["F_obs"]).to(dev), P4.h, P4.sources)
        phi = torch.empty_like(F)
        g = torch.zeros_like(F)
        dF = torch.empty_like(F)

        def step():
            eik.solve(F, P4.h, P4.sources, out=phi)
            g.view(-1)[rec] = 2 * (phi.view(-1)[rec] - t_obs.view(-1)[rec])
            eik.adjoint(F, phi, P4.h, P4.sources, g, out=dF)
        ms = _gpu_ms(torch, step, steps)
        F64 = P4.F.astype(np.float64)
        t64 = oracle.fmm(P4.meta["F_obs"].astype(np.float64), P4.h, P4.sources).ravel()[P4.receivers]

        def ostep():
            p = oracle.fmm(F64, P4.h, P4.sources)
            go = np.zeros(p.size)
            go[P4.receivers] = 2 * (p.ravel()[P4.receivers] - t64)
            oracle.adjoint(F64, P4.h, P4.sources, p, go.reshape(p.shape))
        med, runs = oracle_time(ostep)
        return {"forward_adjoint": {"ms": ms, "node_updates_per_s": P4.n / (ms / 1e3),
                                    "loss": "sum over 64 bottom-face receivers of (phi - t_obs)^2"},
                "oracle_forward_adjoint": {"ms": med * 1e3, "runs_s": runs, "cores": 1}}

    row("4: 192^3 FP32 layered + anomalies, forward and misfit adjoint", P4, {"tile": dict(variant="tile")},
        fwd_adjoint=misfit)

    b = batch_bench(torch, eik, W, 256, steps)
    Ps = W.batch_2d(256)
    workers = host_cpu()["usable_cpus"] or 1

    def one(P):
        F64 = P.F.astype(np.float64)
        p = oracle.fmm(F64, P.h, P.sources)
        g = np.zeros(P.F.size)
        g[P.receivers] = 1.0
        oracle.adjoint(F64, P.h, P.sources, p, g.reshape(P.F.shape))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(one, Ps))
    wall = time.perf_counter() - t0
    nb = b["config"]["nodes"]
    rows.append({"config": "5: 256 2D FP32 lognormal grids, sides 128..2048, 1-8 sources; forward + adjoint",
                 "nodes": nb,
                 "graph_forward_adjoint": {"ms": b["graph_ms_per_step"], "node_updates_per_s": b["value"]},
                 "eager_forward_adjoint": {"ms": b["eager_ms_per_step"]},
                 "parity_sample": b["parity_sample"], "tile": b["config"]["tile"],
                 "oracle_forward_adjoint": {"ms": wall * 1e3, "node_updates_per_s": nb / wall,
                                            "cores": workers, "runs_s": [wall],
                                            "note": "one run: fast marching + adjoint per grid on a thread pool"}})
    return rows


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {a.gpus}); "
              "the multi-GPU design is described in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)
    import torch
    if a.copy_calibration:
        n = a.copy_calibration << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n}), flush=True)
        return
    import paper_2106_15869_amd as eik
    import workloads as W

    if a.batch:
        print(json.dumps(batch_bench(torch, eik, W, a.batch, a.steps)), flush=True)
        return
    if a.replay:
        print(json.dumps({"metric": "paper replay: solve ms per example, size and schedule", "unit": "ms",
                          "n_gpus": 1, "data": "synthetic (the paper's analytic examples)", "dtype": "f32",
                          "rows": replay(torch, eik, W)}), flush=True)
        return
    if a.configs:
        print(json.dumps({"metric": "solve ms per workload configuration, GPU beside the float64 oracle",
                          "unit": "ms", "n_gpus": 1, "data": "synthetic", "host": host_cpu(),
                          "rows": configs_table(torch, eik, W, max(3, a.steps // 2))}), flush=True)
        return

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    P = W.maze_3d(a.n)
    F = torch.from_numpy(P.F).to(dev)
    phi = torch.empty_like(F)
    stream = torch.cuda.current_stream(dev)
    need = max(eik.eik_workspace_size(P.dims, eik.make_options(eik.EIK_FLOAT32, v)) for v in ("tile", "node", "fim"))
    need = max(need, eik.eik_adjoint_workspace_size(P.dims, eik.make_options(eik.EIK_FLOAT32)))
    ws = torch.empty(need, dtype=torch.uint8, device=dev)

    def fwd(variant=a.variant, **kw):
        return eik.solve(F, P.h, P.sources, variant=variant, out=phi, workspace=ws, stream=stream, **kw)

    # counters of one solve, then the timed region
    _, st = fwd(stats=True)
    ms, wall = timed(torch, fwd, a.steps, a.warmup, stream)
    value = P.n / (ms / 1e3)

    # dominant kernel, timed with HIP events on the library's stream
    _, pst = fwd(stats=True, profile=True)
    kernels = pst["kernels"]
    dom = max(kernels, key=lambda k: kernels[k]["ms"])
    tile_nodes = 8 * 8 * 8
    dom_ms = kernels[dom]["ms"]
    dom_launches = max(kernels[dom]["launches"], 1)
    b_alg = alg_bytes(dom, pst)
    b_staged = staged_bytes(dom, pst, a.variant, P.n, tile_nodes)
    achieved = b_alg / (dom_ms / 1e3) / 1e9 if b_alg else None
    kname = f"{'k_tile_' if a.variant == 'tile' else 'k_'}{dom}"
    ksym = f"{kname}IfLi3ELi8ELi8ELi8ELb0E" if a.variant == "tile" else f"{kname}IfLi3E"
    code_hash = kernel_code_hash(ksym)
    floor = 28 * P.n  # 3 evaluations x 8 B + one 4 B write per node
    roofline = {
        "bound": "hbm",
        "kernel": kname,
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS if achieved else None,
        "traffic": measured_traffic(kname, code_hash),
        "bytes_rule": "8 B per local-solver evaluation (F, phi) + 4 B per changed value",
        "launches": dom_launches,
        "avg_launch_us": dom_ms * 1e3 / dom_launches,
        "algorithmic_bytes_per_launch": b_alg / dom_launches if b_alg else None,
        "kernel_code_sha16": code_hash,
        "staged": {"bytes_per_launch": b_staged / dom_launches if b_staged else None,
                   "achieved_GBs": b_staged / (dom_ms / 1e3) / 1e9 if b_staged else None,
                   "rule": "tile visits x 512 nodes x 9 B (F, phi, label) + changed values x 4 B"},
        "solve_floor": {"bytes": floor, "achieved_GBs": floor / (ms / 1e3) / 1e9,
                        "frac": floor / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                        "rule": "28 B per node: 3 evaluations x 8 B + one 4 B write"},
        "kernel_ms_per_solve": {k: v["ms"] for k, v in kernels.items()},
    }

    out = {
        "metric": "node-updates/s and solve ms, 3D 256^3 FP32, fwd and fwd+adjoint; % HBM peak",
        "value": value,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"maze_3d {a.n}^3: 8^3 obstacle blocks (F=0.001, p=0.3) in F=1, h=1, "
                               "source (0,0,0); forward solve",
                   "schedule": a.variant, "grid": list(P.dims), "nodes": P.n},
        "roofline": roofline,
        "wall_ms_per_step": wall,
        "evaluations_per_s": (st["evals_step2"] + st["evals_early"] + st["evals_detect"] + st["evals_remedy"])
        / (ms / 1e3),
        "evaluations_per_node": {"update": st["evals_step2"] / P.n, "early_remedy": st["evals_early"] / P.n,
                                 "detect": st["evals_detect"] / P.n, "remedy": st["evals_remedy"] / P.n},
        "stats": st,
    }

    if not a.no_extra:
        rec = W.receivers_on_face(P.dims, 64, W.BASE_SEED + 1, axis=0, side=-1)
        g = torch.zeros_like(F)
        g.view(-1)[torch.from_numpy(rec).to(dev)] = 1.0
        dF = torch.empty_like(F)

        def fwd_adj():
            fwd()
            eik.adjoint(F, phi, P.h, P.sources, g, out=dF, workspace=ws, stream=stream)

        ms_fa, _ = timed(torch, fwd_adj, max(1, a.steps // 2), 1, stream)
        out["fwd_adjoint"] = {"ms_per_step": ms_fa, "node_updates_per_s": P.n / (ms_fa / 1e3),
                              "adjoint_ms": ms_fa - ms,
                              "loss": "sum of phi at 64 receivers on the face z = 255"}
        other = "node" if a.variant == "tile" else "tile"
        _, st_o = fwd(variant=other, stats=True)
        ms_o, _ = timed(torch, lambda: fwd(variant=other), max(1, a.steps // 2), 1, stream)
        out["other_schedule"] = {"schedule": other, "ms_per_step": ms_o,
                                 "node_updates_per_s": P.n / (ms_o / 1e3), "stats": st_o}
        # the tile schedule with its remedy run first-in first-out
        _, st_q = fwd(variant="tile", fifo=True, stats=True)
        ms_q, _ = timed(torch, lambda: fwd(variant="tile", fifo=True), max(1, a.steps // 2), 1, stream)
        out["fifo_remedy"] = {"schedule": "tile, remedy first-in first-out", "ms_per_step": ms_q,
                              "node_updates_per_s": P.n / (ms_q / 1e3), "stats": st_q}
        # the method the paper improves on, on the same node lists and GPU
        _, st_f = fwd(variant="fim", stats=True)
        ms_f, _ = timed(torch, lambda: fwd(variant="fim"), max(1, a.steps // 5), 1, stream)
        out["fim_baseline"] = {"schedule": "fim (node lists, neighbour check, no remedy)",
                               "ms_per_step": ms_f, "node_updates_per_s": P.n / (ms_f / 1e3),
                               "stats": st_f}
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(P)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
