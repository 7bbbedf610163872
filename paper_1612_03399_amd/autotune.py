"""Launch-shape autotuner of the fused step: a staged search with a cache.

How fast the fused step runs depends on how the batch is cut into work units
(whole bodies, or patches of larger ones), on the workgroup size, on how many
workgroups share a compute unit (which sets the LDS left for each grid tile)
and on the tile cap; the best choice depends on the batch (body sizes, their
extent in cells).  `autotune` searches these ip_plan_options coarse to fine:

1. the workgroup shape: threads x workgroups per compute unit, with the
   default unit split;
2. around the best shape: the unit split (the largest body kept whole,
   `unit_nodes`) and the patch size (`patch_owned`);
3. around the best of those: a cap on the tile region (`tile_bytes`).

Each candidate is a plan with the reference bound, timed over a few steps on
scratch copies of the caller's inputs (the caller's positions and force field
are not touched); candidates that resolve to a launch shape already timed are
skipped, and a later candidate replaces the current choice only when it is
faster by more than the timing noise (`choose`).  Every candidate computes
the same step: the choice changes the speed, not the results beyond
summation order.

The result is cached in a JSON file keyed by the device architecture, a
signature of the workload (body, node, edge and face counts, the histogram of
body sizes, the grid) and the precision, so a second call on the same kind of
batch costs one lookup.  The cache file is $IPIBM_TUNE_CACHE, else
~/.cache/ipibm/autotune.json.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np
import torch

from . import native as N

#: Stage 1: workgroup shapes (threads, workgroups per compute unit); {} is the
#: default split (units above 1536 nodes on 768 threads, the rest on 384, two
#: per compute unit).  128-thread units need small patches for their tiles
#: to fit four or six to a compute unit, so those shapes come with their
#: patch size.
STAGE1 = (
    {},
    {"threads": 768},
    {"threads": 384},
    {"threads": 384, "wg_per_cu": 2},
    {"threads": 256, "wg_per_cu": 2},
    {"threads": 256, "wg_per_cu": 3},
    {"threads": 128, "wg_per_cu": 4, "patch_owned": 256},
    {"threads": 128, "wg_per_cu": 6, "patch_owned": 128},
)
#: Stage 2: unit splits tried on the best stage-1 shape.
STAGE2 = (
    {"unit_nodes": 384},
    {"unit_nodes": 768},
    {"patch_owned": 256},
    {"patch_owned": 384},
    {"patch_owned": 768},
    {"unit_nodes": 768, "patch_owned": 256},
)
#: Stage 3: tile caps tried on the best stage-2 choice.
STAGE3 = (
    {"tile_bytes": 16384},
    {"tile_bytes": 32768},
)


def time_plan(plan, X, ref, k, u, dt, steps=5, warmup=2, f=None):
    """Mean milliseconds of ip_step over `steps` after `warmup`, on scratch
    copies (the plan must have the reference bound)."""
    Xs = X.clone()
    fs = torch.zeros_like(u) if f is None else f
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        N.ip_step(plan, Xs, None, k, u, fs, dt, stream=stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        N.ip_step(plan, Xs, None, k, u, fs, dt, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    code, flags = N.ip_plan_status(plan)
    if code != N.IP_OK:
        raise N.IpibmError(code, f"device status {flags} while timing options {plan.options}")
    return e0.elapsed_time(e1) / steps


def choose(results, margin=0.02):
    """The result to keep: candidates are listed in order of preference, and
    a later one replaces the current choice only when it is faster by more
    than `margin` (the timing noise)."""
    best = results[0]
    for r in results[1:]:
        if r["ms"] < (1.0 - margin) * best["ms"]:
            best = r
    return best


def merged(base, extra):
    out = dict(base)
    out.update(extra)
    return out


def staged_candidates(best1, best2=None):
    """Candidates of stages 2 and 3 around the best of the previous stage."""
    if best2 is None:
        return [merged(best1, c) for c in STAGE2]
    return [merged(best2, c) for c in STAGE3]


def signature(mesh, grid, precision):
    """Workload key: counts, the histogram of body sizes and the grid."""
    no = np.asarray(mesh.node_off, np.int64)
    sizes = np.diff(no)
    vals, counts = np.unique(sizes, return_counts=True)
    h = hashlib.sha1()
    h.update(np.asarray([len(no) - 1, no[-1], np.asarray(mesh.edge_off)[-1],
                         np.asarray(mesh.face_off)[-1]], np.int64).tobytes())
    h.update(vals.astype(np.int64).tobytes())
    h.update(counts.astype(np.int64).tobytes())
    h.update(np.asarray([grid.nx, grid.ny, grid.nz], np.int64).tobytes())
    h.update(np.asarray([float(grid.h)]).tobytes())
    h.update(precision.encode())
    return h.hexdigest()[:20]


def arch():
    try:
        return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def cache_path():
    return os.environ.get("IPIBM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "ipibm", "autotune.json"))


def cache_key(mesh, grid, precision):
    return f"{arch()}|{signature(mesh, grid, precision)}|{precision}"


def cache_load():
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def cache_store(key, entry):
    data = cache_load()
    data[key] = entry
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_candidates(mesh, grid, precision, X, ref, k, u, dt, candidates, steps, warmup, seen,
                     Xref, f, stage, results):
    for opt in candidates:
        plan = N.Plan(mesh, grid, precision, opt)
        try:
            if ref[0] is None:
                ref[0] = N.ip_reference_from(plan, Xref)
            shape = (plan.fused, plan.n_units, plan.step_threads, plan.tile_bytes,
                     plan.largest_unit)
            if shape in seen:          # resolves to a launch shape already timed
                continue
            seen.add(shape)
            N.ip_plan_bind_reference(plan, ref[0])
            ms = time_plan(plan, X, ref[0], k, u, dt, steps, warmup, f)
            results.append({"options": dict(opt), "ms": ms, "stage": stage, "fused": plan.fused,
                            "units": plan.n_units, "threads": plan.step_threads,
                            "tile_bytes": plan.tile_bytes, "largest_unit": plan.largest_unit})
        finally:
            plan.close()


def autotune(mesh, grid, precision, X, ref, k, u, dt, steps=5, warmup=2, Xref=None,
             use_cache=True, stages=(STAGE1,)):
    """Returns (best options dict, list of per-candidate results, info).

    `ref` is a native.Reference of the mesh (caller's element order), or None
    with the reference positions `Xref` given (the reference is then computed
    once, with the first candidate's plan); X, u on the device.  `stages[0]`
    lists the stage-1 shapes.  info = {"cache": "hit" | "miss" | "off",
    "key", "seconds"}; on a hit the results list is the cached search."""
    t0 = time.perf_counter()
    key = cache_key(mesh, grid, precision)
    if use_cache:
        hit = cache_load().get(key)
        if hit is not None:
            return dict(hit["options"]), hit["results"], {
                "cache": "hit", "key": key, "seconds": time.perf_counter() - t0,
                "path": cache_path()}
    results, seen, refbox = [], set(), [ref]
    f = torch.zeros_like(u)
    _time_candidates(mesh, grid, precision, X, refbox, k, u, dt, stages[0], steps, warmup, seen,
                     Xref, f, 1, results)
    best1 = choose(results)["options"]
    _time_candidates(mesh, grid, precision, X, refbox, k, u, dt, staged_candidates(best1), steps,
                     warmup, seen, Xref, f, 2, results)
    best2 = choose(results)["options"]
    _time_candidates(mesh, grid, precision, X, refbox, k, u, dt, staged_candidates(best1, best2),
                     steps, warmup, seen, Xref, f, 3, results)
    best = choose(results)["options"]
    info = {"cache": "miss" if use_cache else "off", "key": key,
            "seconds": time.perf_counter() - t0}
    if use_cache:
        cache_store(key, {"options": best, "results": results, "searched": time.time()})
        info["path"] = cache_path()
    return dict(best), results, info
