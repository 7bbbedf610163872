"""Launch-shape autotuner of the fused step.

How fast the fused step runs depends on how the batch is cut into work units
(whole bodies, or patches of larger ones), on the workgroup size and on the
LDS given to the grid tile; the best choice depends on the batch (body sizes,
their extent in cells).  `autotune` builds a plan for each candidate
ip_plan_options, binds the reference, times a few steps on scratch copies of
the caller's inputs (the caller's positions and force field are not touched),
checks that every step ended without a device status, and returns the fastest
options together with all timings.  Every candidate computes the same step:
the choice changes the speed, not the results beyond summation order.
"""
from __future__ import annotations

import torch

from . import native as N

#: Candidate launch shapes: 768 threads with whole bodies up to 3072 nodes,
#: the same with a capped tile, 384 threads (units up to 1536 nodes, two
#: workgroups per compute unit when their LDS fits), 384 threads with small
#: patches and a capped tile (more, smaller units sharing compute units), and
#: bodies above 768 or 1536 nodes cut into patches of 256 or 512 owned nodes
#: (bodies that span many cells get patches whose grid tiles fit LDS).
CANDIDATES = (
    {},
    {"threads": 768, "tile_bytes": 32768},
    {"threads": 384},
    {"threads": 384, "unit_nodes": 768, "patch_owned": 512, "tile_bytes": 16384},
    {"threads": 384, "unit_nodes": 640, "patch_owned": 384, "tile_bytes": 12288},
    {"unit_nodes": 768, "patch_owned": 256},
    {"unit_nodes": 1536, "patch_owned": 512},
)

#: A shorter list for large batches of uneven bodies, where building each
#: plan costs seconds: the default, one workgroup per compute unit with the
#: largest tiles, and small patches two per compute unit.
UNEVEN_CANDIDATES = (
    {},
    {"threads": 384},
    {"unit_nodes": 768, "patch_owned": 256},
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


def autotune(mesh, grid, precision, X, ref, k, u, dt, candidates=CANDIDATES, steps=5, warmup=2,
             Xref=None):
    """Returns (best options dict, list of per-candidate results).  `ref` is a
    native.Reference of the mesh (caller's element order), or None with the
    reference positions `Xref` given (the reference is then computed once,
    with the first candidate's plan); X, u on the device."""
    results = []
    seen = set()
    f = torch.zeros_like(u)
    for opt in candidates:
        plan = N.Plan(mesh, grid, precision, opt)
        try:
            if ref is None:
                ref = N.ip_reference_from(plan, Xref)
            shape = (plan.fused, plan.n_units, plan.step_threads, plan.tile_bytes,
                     plan.largest_unit)
            if shape in seen:          # resolves to a launch shape already timed
                continue
            seen.add(shape)
            N.ip_plan_bind_reference(plan, ref)
            ms = time_plan(plan, X, ref, k, u, dt, steps, warmup, f)
            results.append({"options": dict(opt), "ms": ms, "fused": plan.fused,
                            "units": plan.n_units, "threads": plan.step_threads,
                            "tile_bytes": plan.tile_bytes, "largest_unit": plan.largest_unit})
        finally:
            plan.close()
    return choose(results)["options"], results


def choose(results, margin=0.02):
    """The result to keep: candidates are listed in order of preference, and
    a later one replaces the current choice only when it is faster by more
    than `margin` (the timing noise)."""
    best = results[0]
    for r in results[1:]:
        if r["ms"] < (1.0 - margin) * best["ms"]:
            best = r
    return best
