#!/usr/bin/env python3
"""Benchmark: IFIM eikonal solve, 3D 256^3 float32 maze, one MI355X.

One step = one complete solve (initialisation, update step, remedy step) of
the 256^3 maze workload: blocks of 8^3 cells are obstacles (F = 0.001) with
probability 0.3, else free (F = 1); h = 1; source at (0,0,0) with its block
forced free.  Inputs are resident in HBM before the timed region; the
workspace is preallocated.  value = grid nodes solved per second.

Prints ONE JSON line (rank 0).  --gpus N with N > 1 exits: this build runs on
a single GPU.
"""

from __future__ import annotations

import argparse
import json
import os
import subprocess
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
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary variant timing")
    return ap.parse_args()


def time_solves(eik, torch, F, P, variant, steps, warmup, phi, ws, stream):
    for _ in range(warmup):
        eik.solve(F, P.h, P.sources, variant=variant, out=phi, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        eik.solve(F, P.h, P.sources, variant=variant, out=phi, workspace=ws, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    ms = e0.elapsed_time(e1) / steps
    return ms, wall


def cpu_baseline(P):
    import oracle
    F64 = P.F.astype(np.float64)
    t0 = time.perf_counter()
    oracle.fmm(F64, P.h, P.sources)
    dt = time.perf_counter() - t0
    return {"value": P.n / dt, "unit": "node-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"one full {P.name} solve by the float64 fast-marching oracle "
                      f"(single thread, {dt:.1f} s)"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {a.gpus}); "
              "the multi-GPU design is described but not built", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2106_15869_amd as eik
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    P = W.maze_3d(a.n)
    F = torch.from_numpy(P.F).to(dev)
    phi = torch.empty_like(F)
    stream = torch.cuda.current_stream(dev)
    need = max(eik.eik_workspace_size(P.dims, eik.make_options(eik.EIK_FLOAT32, v))
               for v in ("tile", "node"))
    ws = torch.empty(need, dtype=torch.uint8, device=dev)

    # one solve for the work counters
    _, st = eik.solve(F, P.h, P.sources, variant=a.variant, out=phi, workspace=ws, stats=True)
    ms, wall = time_solves(eik, torch, F, P, a.variant, a.steps, a.warmup, phi, ws, stream)
    value = P.n / (ms / 1e3)

    extra = {}
    if not a.no_extra:
        other = "node" if a.variant == "tile" else "tile"
        try:
            _, st_o = eik.solve(F, P.h, P.sources, variant=other, out=phi, workspace=ws, stats=True)
            ms_o, _ = time_solves(eik, torch, F, P, other, max(1, a.steps // 2), 1, phi, ws, stream)
            extra[other] = {"ms_per_solve": ms_o, "node_updates_per_s": P.n / (ms_o / 1e3),
                            "stats": st_o}
        except Exception as e:  # report, never hide
            extra[other] = {"error": str(e)}

    evals = st["evals_step2"] + st["evals_detect"] + st["evals_remedy"]
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
        "config": {"workload": f"maze_3d_{a.n}^3 (8^3 obstacle blocks F=0.001 p=0.3, F=1 else; "
                               "h=1; source (0,0,0)); forward solve",
                   "variant": a.variant, "grid": list(P.dims), "nodes": P.n},
        "wall_ms_per_step": wall,
        "evaluations_per_s": evals / (ms / 1e3),
        "stats": st,
        "other_variants": extra,
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(P)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
