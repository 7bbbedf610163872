"""Throughput of the IP+IBM Lagrangian step on one MI355X.

A step is one pass of the whole forward hot path over the batch: the four
interaction-potential families with the per-body volume and area reductions,
the gather into nodes, interpolation of the staggered velocity, spreading of
the nodal forces and the explicit update.  Workload: 1000 level-4 icosphere
drops (2 562 000 nodes) on a 256^3 MAC grid, FP64, synthetic seeded inputs
resident in HBM before the timed region.

Prints ONE JSON line (see the metric contract in the design notes).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, published


def touched_points(X, grid):
    """Number of distinct (lattice, point) pairs in the union of all nodes'
    3x3x3 supports (what interpolation reads and spreading updates)."""
    total = 0
    n = np.array([grid.nx, grid.ny, grid.nz], np.int64)
    for d in range(3):
        off = np.array([0.5, 0.5, 0.5])
        off[d] = 0.0
        c = np.floor(X / grid.h - off + 0.5).astype(np.int64)
        keys = []
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    idx = (c + np.array([dx, dy, dz])) % n
                    keys.append((idx[:, 2] * n[1] + idx[:, 1]) * n[0] + idx[:, 0])
        total += np.unique(np.concatenate(keys)).size
    return total


def algorithmic_bytes(wl, touched, real_bytes):
    """Bytes one fused step must move at minimum: X read + write, the
    connectivity and reference arrays as the API holds them, the pinned mask,
    per-body arrays, u read and f read-modify-write over the touched set."""
    N, E, F, B = wl.n_nodes, wl.n_edges, wl.n_faces, wl.n_bodies
    nodes = N * (8 * 3 * 2 + 1)                      # X r+w (FP64), pinned
    edges = E * (16 + real_bytes * 3)                # edges4, l0, cs0[2]
    faces = F * (12 + real_bytes)                    # faces, A0
    bodies = B * 8 * (5 + 1 + 2) + B * (1 + 8 * 3)   # k's+mass, V0, V/A out, closed, offsets
    grid = touched * real_bytes * 3                  # u read, f read + write
    return nodes + edges + faces + bodies + grid


def cpu_baseline(wl, u, budget_s=20.0):
    """The FP64 oracle (single thread, as it stands) on a bounded sample of the
    same workload: whole-batch steps until ~budget_s of CPU work."""
    import oracle as O
    ref = O.reference(wl)
    f = np.zeros_like(u)
    X = wl.X.copy()
    steps = 0
    t0 = time.perf_counter()
    while True:
        X = O.step(wl, X, ref, u, wl.dt, f)["X"]
        steps += 1
        el = time.perf_counter() - t0
        if el > budget_s / 2 or steps >= 3:
            break
    return {"value": wl.n_nodes * steps / el, "unit": "node-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{steps} full step(s) of the {wl.n_bodies}-body batch "
                      f"({wl.n_nodes} nodes), {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--bodies", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is described in the design notes, not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1612_03399_amd import native as N
    from paper_1612_03399_amd import workload as W

    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    dev = "cuda:0"
    torch.cuda.set_device(0)
    wl = W.config1(n_bodies=args.bodies, precision=args.precision)
    log(f"workload {wl.name}: {wl.n_nodes} nodes, {wl.n_edges} edges, {wl.n_faces} faces")
    u_host = wl.velocity(dtype=np.float64)
    rdt = N.real_dtype(args.precision)
    u = torch.as_tensor(u_host).to(dev, rdt)
    plan = N.Plan(wl, wl.grid, args.precision)
    ref = N.ip_reference_from(plan, torch.as_tensor(wl.Xref).to(dev))
    k = N.Constants.from_arrays(wl.ks, wl.kb, wl.kA, wl.kV, wl.mass, dev)
    X = torch.as_tensor(wl.X).to(dev)
    f = torch.zeros(u.shape, dtype=rdt, device=dev)
    V = torch.empty(wl.n_bodies, dtype=torch.float64, device=dev)
    A = torch.empty_like(V)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        N.ip_step(plan, X, ref, k, u, f, wl.dt, V, A, stream)
    torch.cuda.synchronize()
    code, flags = N.ip_plan_status(plan)
    if code != N.IP_OK:
        raise SystemExit(f"device status {code} flags {flags}")
    log(f"warmup done ({args.warmup} steps)")

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        N.ip_step(plan, X, ref, k, u, f, wl.dt, V, A, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    log(f"timed {args.steps} steps: {ms:.4f} ms/step")

    real_bytes = 8 if args.precision == "f64" else 4
    touched = touched_points(wl.X, wl.grid)
    bytes_step = algorithmic_bytes(wl, touched, real_bytes)
    gbs = bytes_step / (ms * 1e-3) / 1e9
    value = wl.n_nodes / (ms * 1e-3)

    out = {
        "metric": "Lagrangian node-steps/s (forces+interp+spread+update)",
        "value": value, "unit": "node-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.precision,
        "data": "synthetic (seeded icosphere drops, random-Fourier MAC velocity)",
        "config": {"workload": wl.name, "bodies": wl.n_bodies, "nodes": wl.n_nodes,
                   "edges": wl.n_edges, "faces": wl.n_faces,
                   "grid": [wl.grid.nx, wl.grid.ny, wl.grid.nz], "dt": wl.dt},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "whole step", "bytes_per_step": bytes_step,
                     "bytes_per_node": bytes_step / wl.n_nodes, "touched_grid_points": touched},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(wl, u_host)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
