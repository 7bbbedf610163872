"""Throughput of the IP+IBM Lagrangian step on one MI355X.

A step is one pass of the whole forward hot path over the batch: the four
interaction-potential families with the per-body volume and area reductions,
the accumulation into nodes, interpolation of the staggered velocity,
spreading of the nodal forces and the explicit update.  The default workload
is 1000 level-4 icosphere drops (2 562 000 nodes) on a 256^3 MAC grid in FP64,
synthetic seeded inputs resident in HBM before the timed region.  With the
fused path the step is one kernel launch (k_step_fused).  The headline times
a hipGraph of K captured steps, replayed once between HIP events on the
stream the kernels run on (after W eager warm-up steps and one untimed
replay); the same K steps launched eagerly are reported beside it.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, published
KERNEL_SOURCES = ["paper_1612_03399_amd/csrc/k_step.hip", "paper_1612_03399_amd/csrc/step_common.h",
                  "paper_1612_03399_amd/csrc/elements.h",
                  "paper_1612_03399_amd/csrc/ipibm_internal.h",
                  "paper_1612_03399_amd/csrc/workunits.hip"]
# the reverse step's counters depend on its own kernel too
REVERSE_SOURCES = KERNEL_SOURCES + ["paper_1612_03399_amd/csrc/k_backward.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_{kernel}_{workload}_{dtype}.json")
VALU_FILE = os.path.join(ROOT, "profiles", "valu_k_step_fused_{workload}_{dtype}.json")
# VALU issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction per
# SIMD every 4 cycles (16 lanes per cycle)
VALU_PEAK_WAVE_INSTS = 256 * 4 * 2.4e9 / 4


def kernel_source_hash(sources=KERNEL_SOURCES):
    h = hashlib.sha1()
    for p in sources:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


MAC_OFFSETS = ((0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0))


def touched_points(X, grid, offsets=MAC_OFFSETS):
    """Number of distinct (lattice, point) pairs in the union of all nodes'
    3x3x3 supports (what interpolation reads and spreading updates) over the
    lattices with the given offsets (in cells; default the three MAC ones)."""
    total = 0
    n = np.array([grid.nx, grid.ny, grid.nz], np.int64)
    for off in offsets:
        off = np.asarray(off, np.float64)
        c = np.floor(X / grid.h - off + 0.5).astype(np.int64)
        keys = []
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    idx = (c + np.array([dx, dy, dz])) % n
                    keys.append((idx[:, 2] * n[1] + idx[:, 1]) * n[0] + idx[:, 0])
        total += np.unique(np.concatenate(keys)).size
    return total


def touched_points_device(X, grid, offsets=MAC_OFFSETS, device="cuda"):
    """touched_points() with torch on `device` (for batches of millions of
    nodes): a boolean mask per lattice, set at every support point."""
    import torch
    Xt = torch.as_tensor(np.ascontiguousarray(X, np.float64), device=device)
    n = torch.tensor([grid.nx, grid.ny, grid.nz], dtype=torch.int64, device=device)
    total = 0
    for off in offsets:
        c = torch.floor(Xt / grid.h - torch.tensor(off, dtype=torch.float64, device=device)
                        + 0.5).to(torch.int64)
        mask = torch.zeros(grid.nx * grid.ny * grid.nz, dtype=torch.bool, device=device)
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    i = torch.remainder(c + torch.tensor([dx, dy, dz], device=device), n)
                    mask[(i[:, 2] * n[1] + i[:, 1]) * n[0] + i[:, 0]] = True
        total += int(mask.sum().item())
        del mask, c
    return total


def roofline_block(bytes_per_launch, ms, kernel, extra=None):
    """The roofline object of one leg: algorithmic bytes of one launch over its
    measured duration, against the HBM peak."""
    gbs = bytes_per_launch / (ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": gbs / HBM_PEAK_GBS, "traffic": None, "kernel": kernel,
           "algorithmic_bytes_per_launch": int(bytes_per_launch), "ms_per_launch": ms}
    if extra:
        out.update(extra)
    return out


def reverse_bytes(wl, touched):
    """Bytes one reverse step (k_step_vjp_fused, FP64) must move: X read,
    the incoming adjoint read and the outgoing one written, the pinned mask,
    the packed element records, per-body arrays with the constants' gradients,
    and over the touched grid values u read and the velocity gradient read,
    added to and written."""
    N, E, F, B = wl.n_nodes, wl.n_edges, wl.n_faces, wl.n_bodies
    nodes = N * (8 * 3 * 3 + 1)
    edges = E * 32
    faces = F * 16
    bodies = B * (8 * 8 + 1 + 8 * 3 + 8 * 4)
    grid = touched * 8 * 3
    return nodes + edges + faces + bodies + grid


def algorithmic_bytes(wl, touched, real_bytes):
    """Bytes one step must move at minimum, in the layout the step reads with a
    bound reference: X read + write (FP64), pinned mask, the packed element
    records (four 16-bit local node ids with l0, cos and sin theta0 per edge:
    32 B in FP64, 24 B in FP32; three ids with A0 per face: 16 B), per-body
    arrays, u read and f read-modify-write over the touched grid points."""
    N, E, F, B = wl.n_nodes, wl.n_edges, wl.n_faces, wl.n_bodies
    nodes = N * (8 * 3 * 2 + 1)
    edges = E * (32 if real_bytes == 8 else 24)
    faces = F * 16
    bodies = B * (8 * 8 + 1 + 8 * 3)      # ks kb kA kV mass V0 V A, closed, offsets
    grid = touched * real_bytes * 3       # u read, f read + write
    return nodes + edges + faces + bodies + grid


def load_traffic(workload, dtype, launch, kernel="k_step_fused", sources=KERNEL_SOURCES):
    """Measured HBM bytes per launch from the committed counter summary, when it
    was taken on the current kernel sources and launch shape (else None)."""
    path = TRAFFIC_FILE.format(kernel=kernel, workload=workload, dtype=dtype)
    if not os.path.exists(path):
        return None, None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_hash") != kernel_source_hash(sources):
        return None, "stale (kernel changed since the counters were taken)"
    if t.get("launch") != launch:
        return None, f"taken with launch shape {t.get('launch')}, not {launch}"
    return t["bytes_per_launch"], os.path.relpath(path, ROOT)


def load_valu(workload, dtype, launch, ms):
    """VALU issue of the step from the committed SQ counter record (taken on
    the current kernel sources and launch shape), against the issue peak."""
    path = VALU_FILE.format(workload=workload, dtype=dtype)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_hash") != kernel_source_hash() or t.get("launch") != launch:
        return None
    per_s = t["sq_insts_valu_per_launch"] / (ms * 1e-3)
    return {"wave_instructions_per_launch": t["sq_insts_valu_per_launch"],
            "fp64_wave_instructions_per_launch": t["sq_insts_valu_fp64_per_launch"],
            "achieved_per_s": per_s, "peak_per_s": VALU_PEAK_WAVE_INSTS,
            "frac": per_s / VALU_PEAK_WAVE_INSTS, "source": os.path.relpath(path, ROOT)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_POOL = {}


def _oracle_worker(w, ids, shm_name, shape, barrier, go, done):
    """One process of the parallel oracle: steps its bodies of the batch
    (the oracle unchanged) into its own force field, then adds slab w of
    every process's field into field 0."""
    from multiprocessing import shared_memory
    import oracle as O
    from paper_1612_03399_amd import workload as W
    wl, u = _POOL["wl"], _POOL["u"]
    P = len(_POOL["parts"])
    shm = shared_memory.SharedMemory(name=shm_name)
    fs = np.ndarray((P,) + shape, dtype=np.float64, buffer=shm.buf)
    sub = W.subset(wl, ids)
    ref = O.reference(sub)
    X = sub.X.copy()
    fs[w][...] = 0.0
    barrier.wait(timeout=600)           # set-up done
    go.wait()
    O.step(sub, X, ref, u, wl.dt, fs[w])
    barrier.wait(timeout=600)           # every field complete
    nz = shape[1]
    z0, z1 = w * nz // P, (w + 1) * nz // P
    for q in range(1, P):
        fs[0][:, z0:z1] += fs[q][:, z0:z1]
    barrier.wait(timeout=600)
    del fs
    shm.close()
    done.set()


def cpu_baseline(wl, u, log, single_budget_s=12.0):
    """The FP64 oracle as it stands, timed on the host: one thread on whole
    steps of the batch, and every core available to this process (at most 16)
    with the bodies split into contiguous ranges, one process per range
    calling the unchanged oracle on its bodies, then summing the per-process
    force fields slab by slab (part of the timed step)."""
    import multiprocessing as mp
    from multiprocessing import shared_memory
    import oracle as O
    ref = O.reference(wl)
    f1 = np.zeros_like(u)            # the first step's field, for the parallel run's check
    f2 = np.zeros_like(u)
    X = wl.X.copy()
    steps = 0
    t0 = time.perf_counter()
    while True:
        X = O.step(wl, X, ref, u, wl.dt, f1 if steps == 0 else f2)["X"]
        steps += 1
        el1 = time.perf_counter() - t0
        if el1 > single_budget_s / 2 or steps >= 3:
            break
    single = wl.n_nodes * steps / el1
    log(f"cpu baseline, 1 thread: {steps} step(s) in {el1:.1f} s = {single:.3e} node-steps/s")
    cores = max(1, min(len(os.sched_getaffinity(0)), 16, wl.n_bodies))
    out = {"value": single, "unit": "node-steps/s", "cores": 1, "kind": "oracle",
           "sample": f"{steps} full step(s) of the {wl.n_bodies}-body batch "
                     f"({wl.n_nodes} nodes), {el1:.1f} s on 1 thread",
           "single_thread_value": single, "cpu_model": cpu_model()}
    if cores < 2:
        return out
    P = cores
    sizes = np.diff(np.asarray(wl.node_off))
    cut = np.searchsorted(np.cumsum(sizes), np.arange(1, P) * sizes.sum() / P)
    parts = [p.tolist() for p in np.split(np.arange(wl.n_bodies), cut) if len(p)]
    P = len(parts)
    shape = u.shape
    shm = shared_memory.SharedMemory(create=True, size=P * u.nbytes)
    try:
        _POOL.update(wl=wl, u=u, parts=parts)
        ctx = mp.get_context("fork")
        barrier, go = ctx.Barrier(P + 1), ctx.Event()
        dones = [ctx.Event() for _ in range(P)]
        procs = [ctx.Process(target=_oracle_worker, args=(w, parts[w], shm.name, shape, barrier,
                                                          go, dones[w]))
                 for w in range(P)]
        for pr in procs:
            pr.start()
        try:
            barrier.wait(timeout=600)   # every process has its bodies and reference
            t0 = time.perf_counter()
            go.set()
            barrier.wait(timeout=600)   # fields done
            barrier.wait(timeout=600)   # fields summed
            elp = time.perf_counter() - t0
        except Exception as e:          # a process failed: report the one-thread figure
            for pr in procs:
                pr.terminate()
            for pr in procs:
                pr.join()
            log(f"cpu baseline: parallel oracle failed ({type(e).__name__}); 1 thread only")
            return out
        for pr in procs:
            pr.join()
        fs = np.ndarray((P,) + shape, dtype=np.float64, buffer=shm.buf)
        check = float(np.abs(fs[0] - f1).max() / max(np.abs(f1).max(), 1e-300))
        del fs
    finally:
        _POOL.clear()
        shm.close()
        shm.unlink()
    par = wl.n_nodes / elp
    log(f"cpu baseline, {P} processes: 1 step in {elp:.2f} s = {par:.3e} node-steps/s")
    out.update({"value": par, "cores": P,
                "sample": f"1 full step of the {wl.n_bodies}-body batch ({wl.n_nodes} nodes) "
                          f"on {P} processes (bodies split in {P} ranges, force fields summed "
                          f"by slab), {elp:.2f} s; and {steps} step(s) on 1 thread, {el1:.1f} s",
                "parallel_value": par, "parallel_seconds": elp,
                "parallel_field_rel_diff": check})
    return out


def time_steps(N, plan, X, ref, k, u, f, dt, V, A, steps, warmup, stream, torch):
    for _ in range(warmup):
        N.ip_step(plan, X, ref, k, u, f, dt, V, A, stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        N.ip_step(plan, X, ref, k, u, f, dt, V, A, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def time_graph(N, plan, X, ref, k, u, f, dt, V, A, steps, warmup, torch):
    """W eager warm-up steps, a hipGraph of `steps` captured steps replayed
    once untimed, then once between HIP events on the replay stream."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        N.ip_step(plan, X, ref, k, u, f, dt, V, A, stream)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(steps):
            N.ip_step(plan, X, ref, k, u, f, dt, V, A, torch.cuda.current_stream())
    g.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    del g
    return e0.elapsed_time(e1) / steps


def backward_leg(N, W, bodies, dev, torch, log, steps=10, reps=3):
    """Differentiation workload: the same suspension, loss = sum_b (D_b - D*_b)^2
    on the Taylor deformation after 10 steps, D* ~ U[0.05, 0.2]; gradients with
    respect to X0, u and the per-body constants by the reverse pass over
    checkpoints.  Times the forward (steps + checkpoint copies + loss) and the
    backward separately."""
    from paper_1612_03399_amd import autograd as AG
    wl = W.config4(n_bodies=bodies)
    u = torch.as_tensor(wl.velocity(dtype=np.float64)).to(dev)
    plan = N.Plan(wl, wl.grid, "f64")
    N.ip_plan_bind_reference(plan, N.ip_reference_from(plan, torch.as_tensor(wl.Xref).to(dev)))
    ref = None            # the bound reference (packed once)
    km = torch.as_tensor(np.stack([wl.ks, wl.kb, wl.kA, wl.kV])).to(dev)
    mass = torch.as_tensor(np.asarray(wl.mass, np.float64)).to(dev)
    Ds = torch.as_tensor(wl.targets).to(dev)
    X0 = torch.as_tensor(wl.X).to(dev)
    fwd, bwd = [], []
    for r in range(reps + 1):
        x0 = X0.clone().requires_grad_(True)
        uu = u.clone().requires_grad_(True)
        kk = km.clone().requires_grad_(True)
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        torch.cuda.synchronize()
        e[0].record()
        loss = AG.taylor_loss(plan, AG.rollout(plan, x0, uu, kk, ref, mass, wl.dt, steps), Ds)
        e[1].record()
        loss.backward()
        e[2].record()
        torch.cuda.synchronize()
        if r > 0:                       # the first pass allocates the workspace
            fwd.append(e[0].elapsed_time(e[1]))
            bwd.append(e[1].elapsed_time(e[2]))
    f, b = float(np.median(fwd)), float(np.median(bwd))
    log(f"backward leg: fwd {f:.3f} ms, bwd {b:.3f} ms for {steps} steps (ratio {b / f:.2f})")
    # the reverse-step kernel alone: one ip_step_vjp per step, against one
    # forward ip_step, each timed over `kreps` back-to-back calls
    k = N.Constants.from_arrays(wl.ks, wl.kb, wl.kA, wl.kV, wl.mass, dev)
    X = X0.clone()
    lam = torch.randn(X.shape, dtype=torch.float64, device=dev, generator=torch.Generator(
        device=dev).manual_seed(1004))
    lam2 = torch.empty_like(lam)
    gk = torch.zeros(4, wl.n_bodies, dtype=torch.float64, device=dev)
    gu = torch.zeros_like(u)
    stream = torch.cuda.current_stream()
    kreps = 20

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(kreps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / kreps

    t_rev = timed(lambda: N.ip_step_vjp(plan, X, ref, k, u, wl.dt, lam, lam2, gk, gu,
                                        stream=stream))
    f_grid = torch.zeros_like(u)
    Xf = X0.clone()
    t_fwd = timed(lambda: N.ip_step(plan, Xf, ref, k, u, f_grid, wl.dt, stream=stream))
    code, flags = N.ip_plan_status(plan)
    if code != N.IP_OK:
        raise SystemExit(f"device status {code} flags {flags} in the backward leg")
    touched = touched_points_device(wl.X, wl.grid, device=dev)
    rb = reverse_bytes(wl, touched)
    log(f"reverse step kernel: {t_rev:.4f} ms against {t_fwd:.4f} ms forward "
        f"({t_rev / t_fwd:.2f}x), {rb / (t_rev * 1e-3) / (HBM_PEAK_GBS * 1e9):.1%} of HBM")
    launch = {"threads": plan.step_threads, "tile_bytes": plan.tile_bytes, "units": plan.n_units}
    rr = roofline_block(rb, t_rev, f"k_step_vjp_fused<{plan.step_threads}, false>",
                        {"touched_grid_points": touched, "launch": launch})
    traffic, traffic_src = load_traffic(wl.name, "f64", launch, kernel="k_step_vjp_fused",
                                        sources=REVERSE_SOURCES)
    if traffic is not None:
        rr.update({"traffic": traffic, "traffic_source": traffic_src})
    elif traffic_src is not None:
        rr["traffic_note"] = traffic_src
    out = {"diff_workload": wl.name, "diff_steps": steps, "diff_fwd_ms": f, "diff_bwd_ms": b,
           "diff_bwd_over_fwd": b / f, "diff_loss": float(loss.item()),
           "reverse_step_ms": t_rev, "forward_step_ms": t_fwd,
           "reverse_over_forward_step": t_rev / t_fwd,
           "reverse_roofline": rr}
    del plan, X, Xf, lam, lam2, gk, gu, f_grid, u
    torch.cuda.empty_cache()
    return out


def uneven_leg(N, W, dev, torch, log, steps=10, sample=256):
    """The uneven batch (4096 bodies of levels 2-5, 512^3, FP32 forces and
    grid): the batched step (one fused launch over all work units), the same
    captured in a hipGraph and replayed, and plain per-body launches (one plan
    and one ip_step per body) against the batched step on a seeded sample of
    the bodies.  The velocity is a seeded uniform random field generated on
    the device: the cost does not depend on its values."""
    wl = W.config2()
    log(f"uneven leg: {wl.n_bodies} bodies, {wl.n_nodes} nodes")
    g = torch.Generator(device=dev)
    g.manual_seed(1002)
    u = (torch.rand((3, wl.grid.nz, wl.grid.ny, wl.grid.nx), generator=g, device=dev,
                    dtype=torch.float32) - 0.5) * 0.2
    f = torch.zeros_like(u)
    k = N.Constants.from_arrays(wl.ks, wl.kb, wl.kA, wl.kV, wl.mass, dev)
    X = torch.as_tensor(wl.X).to(dev)
    Xref = torch.as_tensor(wl.Xref).to(dev)
    from paper_1612_03399_amd import autotune as AT
    opts, tuned, tinfo = AT.autotune(wl, wl.grid, "f32", X, None, k, u, wl.dt, Xref=Xref)
    log(f"  uneven autotune: cache {tinfo['cache']} ({tinfo['seconds']:.1f} s)")
    for r in tuned:
        log(f"  uneven options {r['options']}: {r['ms']:.3f} ms ({r['units']} units, "
            f"{r['threads']} threads, tile {r['tile_bytes']} B)")
    plan = N.Plan(wl, wl.grid, "f32", opts)
    ref = N.ip_reference_from(plan, Xref)
    N.ip_plan_bind_reference(plan, ref)
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    batched = timed(lambda: N.ip_step(plan, X, None, k, u, f, wl.dt, stream=stream), steps)
    gr = torch.cuda.CUDAGraph()
    s2 = torch.cuda.Stream()
    s2.wait_stream(stream)
    with torch.cuda.stream(s2):
        N.ip_step(plan, X, None, k, u, f, wl.dt, stream=s2)
    stream.wait_stream(s2)
    torch.cuda.synchronize()
    with torch.cuda.graph(gr):
        for _ in range(10):
            N.ip_step(plan, X, None, k, u, f, wl.dt, stream=torch.cuda.current_stream())
    graph = timed(gr.replay, 3) / 10
    code, flags = N.ip_plan_status(plan)
    if code != N.IP_OK:
        raise SystemExit(f"device status {code} flags {flags} in the uneven leg")
    touched = touched_points_device(wl.X, wl.grid, device=dev)
    ub = algorithmic_bytes(wl, touched, 4)
    # counters of the step kernel alone (the geometry and commit passes of the
    # patched bodies excluded), when taken on these sources and this shape
    launch = {"threads": plan.step_threads, "tile_bytes": plan.tile_bytes, "units": plan.n_units}
    traffic, traffic_src = load_traffic(wl.name, "f32", launch)
    valu = load_valu(wl.name, "f32", launch, graph)
    out = {"uneven_workload": wl.name, "uneven_nodes": wl.n_nodes, "uneven_options": opts,
           "uneven_autotune": [{"options": r["options"], "ms": r["ms"], "stage": r["stage"]}
                               for r in tuned],
           "uneven_autotune_cache": tinfo["cache"],
           "uneven_units": plan.n_units, "uneven_patched_bodies": plan.patched_bodies,
           "uneven_batched_ms": batched, "uneven_graph_ms": graph,
           "uneven_node_steps_per_s": wl.n_nodes / (graph * 1e-3),
           "uneven_roofline": roofline_block(
               ub, graph, "k_step_fused<float, %d, false> + geometry and commit passes"
               % plan.step_threads, {"touched_grid_points": touched,
                                     "bytes_per_node": ub / wl.n_nodes,
                                     "traffic": traffic, "traffic_source": traffic_src,
                                     "traffic_kernel": "k_step_fused only",
                                     "valu_issue": valu})}
    log(f"uneven: {ub / 1e9:.3f} GB algorithmic per step, "
        f"{out['uneven_roofline']['frac']:.1%} of HBM at the graph replay's time")
    del gr, plan
    # per-body launches on a sample, against the batched step of the same bodies
    ids = np.sort(np.random.default_rng(7).choice(wl.n_bodies, sample, replace=False))
    sub = W.subset(wl, ids)
    ks = N.Constants.from_arrays(sub.ks, sub.kb, sub.kA, sub.kV, sub.mass, dev)
    bplan = N.Plan(sub, sub.grid, "f32", opts)
    N.ip_plan_bind_reference(bplan, N.ip_reference_from(bplan, torch.as_tensor(sub.Xref).to(dev)))
    Xs = torch.as_tensor(sub.X).to(dev)
    sample_batched = timed(lambda: N.ip_step(bplan, Xs, None, ks, u, f, wl.dt, stream=stream), steps)
    singles = []
    for b in ids:
        one = W.subset(wl, [b])
        p1 = N.Plan(one, one.grid, "f32")
        N.ip_plan_bind_reference(p1, N.ip_reference_from(p1, torch.as_tensor(one.Xref).to(dev)))
        singles.append((p1, torch.as_tensor(one.X).to(dev),
                        N.Constants.from_arrays(one.ks, one.kb, one.kA, one.kV, one.mass, dev)))

    def per_body():
        for p1, x1, k1 in singles:
            N.ip_step(p1, x1, None, k1, u, f, wl.dt, stream=stream)

    sample_single = timed(per_body, 3)
    for p1, _, _ in singles:
        code, flags = N.ip_plan_status(p1)
        if code != N.IP_OK:
            raise SystemExit(f"device status {code} flags {flags} in a per-body plan")
    out.update({"per_body_sample": int(sample), "per_body_sample_nodes": sub.n_nodes,
                "per_body_sample_ms": sample_single, "batched_sample_ms": sample_batched,
                "per_body_over_batched": sample_single / sample_batched})
    log(f"uneven: batched {batched:.3f} ms, graph {graph:.3f} ms/step; sample of {sample}: "
        f"per-body {sample_single:.3f} ms vs batched {sample_batched:.3f} ms")
    return out


def mls_leg(N, W, bodies, dev, torch, log, reps=20, alpha=0.4):
    """MLS transfer at the triangle centroids on the same batch (one marker per
    face): ibm_interp_mls, ibm_spread_mls, ibm_direct_forcing_mls and
    ibm_probe_loads timed with HIP events on the launch
    stream, and their algorithmic bytes: vertex positions read once, face
    indices, the marker values, and the grid values in the union of the
    markers' 27-point supports (u read; f read and written)."""
    wl = W.config1(n_bodies=bodies)
    log(f"mls leg: {wl.n_faces} markers")
    g = torch.Generator(device=dev)
    g.manual_seed(1001)
    u = (torch.rand((3, wl.grid.nz, wl.grid.ny, wl.grid.nx), generator=g, device=dev,
                    dtype=torch.float64) - 0.5) * 0.2
    f = torch.zeros_like(u)
    Fm = torch.rand((wl.n_faces, 3), generator=g, device=dev, dtype=torch.float64) - 0.5
    plan = N.Plan(wl, wl.grid, "f64")
    X = torch.as_tensor(wl.X).to(dev)
    U = torch.empty(wl.n_faces, 3, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_i = timed(lambda: N.ibm_interp_mls(plan, X, u, alpha, U, stream=stream))
    t_s = timed(lambda: N.ibm_spread_mls(plan, X, Fm, alpha, f, stream=stream))
    # direct forcing (F = (Vb - U)/dt, spread) in one pass, marker forces stored
    Vb = torch.zeros_like(Fm)
    t_d = timed(lambda: N.ibm_direct_forcing_mls(plan, X, Vb, u, alpha, 1e-4, f, Fm=U,
                                                 stream=stream))
    # external loads by normal probes: pressure at cell centres, mu = 1e-3
    p = (torch.rand((wl.grid.nz, wl.grid.ny, wl.grid.nx), generator=g, device=dev,
                    dtype=torch.float64) - 0.5)
    acc = torch.rand((wl.n_faces, 3), generator=g, device=dev, dtype=torch.float64) - 0.5
    t_p = timed(lambda: N.ibm_probe_loads(plan, X, u, p, alpha, 1e-3, acc=acc, Fext=U,
                                          stream=stream))
    code, flags = N.ip_plan_status(plan)
    if code != N.IP_OK:
        raise SystemExit(f"device status {code} flags {flags} in the mls leg")
    fa = np.asarray(wl.faces)
    cen = (wl.X[fa[:, 0]] + wl.X[fa[:, 1]] + wl.X[fa[:, 2]]) / 3.0
    touched = touched_points(cen, wl.grid)
    nrm = np.cross(wl.X[fa[:, 1]] - wl.X[fa[:, 0]], wl.X[fa[:, 2]] - wl.X[fa[:, 0]])
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    ends = [cen + wl.grid.h * nrm]
    closed = np.repeat(np.asarray(wl.closed, bool), np.diff(np.asarray(wl.face_off)))
    if not closed.all():
        ends.append(cen[~closed] - wl.grid.h * nrm[~closed])
    ends = np.concatenate(ends)
    touched_p = touched_points(ends, wl.grid, MAC_OFFSETS + ((0.5, 0.5, 0.5),))
    common = wl.n_nodes * 24 + wl.n_faces * 12
    b_i = common + wl.n_faces * 24 + touched * 8
    b_s = common + wl.n_faces * 24 + touched * 16
    # probes: positions, faces, acc read and Fext written per face, u and p
    # over the union of the probe ends' supports
    b_p = common + wl.n_faces * 48 + touched_p * 8
    out = {"mls_markers": wl.n_faces, "mls_alpha": alpha,
           "probe_loads_ms": t_p, "probe_loads_algorithmic_bytes": b_p,
           "probe_loads_hbm_frac": b_p / (t_p * 1e-3) / (HBM_PEAK_GBS * 1e9),
           "mls_interp_ms": t_i, "mls_spread_ms": t_s, "mls_direct_forcing_ms": t_d,
           "mls_interp_markers_per_s": wl.n_faces / (t_i * 1e-3),
           "mls_interp_algorithmic_bytes": b_i, "mls_spread_algorithmic_bytes": b_s,
           "mls_interp_hbm_frac": b_i / (t_i * 1e-3) / (HBM_PEAK_GBS * 1e9),
           "mls_spread_hbm_frac": b_s / (t_s * 1e-3) / (HBM_PEAK_GBS * 1e9)}
    log(f"mls: interp {t_i:.3f} ms ({out['mls_interp_hbm_frac']:.1%} of HBM), "
        f"spread {t_s:.3f} ms ({out['mls_spread_hbm_frac']:.1%}), "
        f"direct forcing in one pass {t_d:.3f} ms (interp + spread {t_i + t_s:.3f} ms), "
        f"probe loads {t_p:.3f} ms ({out['probe_loads_hbm_frac']:.1%})")
    del plan, u, f, Fm, U, X, Vb, p, acc
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--bodies", type=int, default=1000)
    ap.add_argument("--workload", default="suspension", choices=["suspension", "uneven"],
                    help="headline batch: the 1000-drop suspension on 256^3 (default) or the "
                         "uneven 4096-body batch on 512^3 (FP32; for its kernel traces and "
                         "counters)")
    ap.add_argument("--options", default=None,
                    help="launch options as JSON (skips the autotuner), e.g. '{\"threads\": 384}'")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other-precision, graph, differentiation and uneven legs")
    ap.add_argument("--legs", default="other,weights,backward,uneven,mls",
                    help="extra legs to run: other (other precision + hipGraph), weights "
                         "(per-edge weights bound), backward, "
                         "uneven, mls (MLS transfer at the triangle centroids)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 512 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "a step sharded over several GPUs is not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1612_03399_amd import autotune as AT
    from paper_1612_03399_amd import native as N
    from paper_1612_03399_amd import workload as W

    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy probe: 512 MiB read + 512 MiB written")

    if args.workload == "uneven":
        wl = W.config2()
        args.precision = "f32"
    else:
        wl = W.config1(n_bodies=args.bodies, precision=args.precision)
    log(f"workload {wl.name}: {wl.n_nodes} nodes, {wl.n_edges} edges, {wl.n_faces} faces")
    u_host = wl.velocity(dtype=np.float64)
    stream = torch.cuda.current_stream()
    k = N.Constants.from_arrays(wl.ks, wl.kb, wl.kA, wl.kV, wl.mass, dev)
    X0 = torch.as_tensor(wl.X).to(dev)

    # launch shape: autotuned on this batch (untimed set-up) unless given; the
    # search is cached, so a second call is a lookup (reported)
    tuning, tune_info = None, None
    if args.options is not None:
        options = json.loads(args.options)
    else:
        rdt = N.real_dtype(args.precision)
        probe = N.Plan(wl, wl.grid, args.precision)
        ref0 = N.ip_reference_from(probe, torch.as_tensor(wl.Xref).to(dev))
        ut = torch.as_tensor(u_host).to(dev, rdt)
        options, tuning, tune_info = AT.autotune(wl, wl.grid, args.precision, X0, ref0, k, ut,
                                                 wl.dt)
        again, _, info2 = AT.autotune(wl, wl.grid, args.precision, X0, ref0, k, ut, wl.dt)
        assert again == options
        tune_info = {"first": tune_info, "second": info2}
        probe.close()
        del ut
        for r in tuning:
            log(f"  options {r['options']}: {r['ms']:.4f} ms ({r['units']} units, "
                f"{r['threads']} threads, tile {r['tile_bytes']} B)")
        log(f"autotuned options: {options} (cache {tune_info['first']['cache']} in "
            f"{tune_info['first']['seconds']:.1f} s, then {tune_info['second']['cache']} in "
            f"{tune_info['second']['seconds'] * 1e3:.1f} ms)")

    def setup(precision):
        rdt = N.real_dtype(precision)
        u = torch.as_tensor(u_host).to(dev, rdt)
        plan = N.Plan(wl, wl.grid, precision, options)
        # the reference is bound once (packed element records); steps pass None
        N.ip_plan_bind_reference(plan, N.ip_reference_from(plan, torch.as_tensor(wl.Xref).to(dev)))
        X = X0.clone()
        f = torch.zeros(u.shape, dtype=rdt, device=dev)
        V = torch.empty(wl.n_bodies, dtype=torch.float64, device=dev)
        A = torch.empty_like(V)
        return plan, None, k, X, u, f, V, A

    plan, ref, k, X, u, f, V, A = setup(args.precision)
    # the same K steps launched eagerly, then as a replayed hipGraph (headline)
    eager_ms = time_steps(N, plan, X, ref, k, u, f, wl.dt, V, A, args.steps, args.warmup,
                          stream, torch)
    ms = time_graph(N, plan, X, ref, k, u, f, wl.dt, V, A, args.steps, args.warmup, torch)
    code, flags = N.ip_plan_status(plan)
    if code != N.IP_OK:
        raise SystemExit(f"device status {code} flags {flags}")
    log(f"timed {args.steps} steps: graph replay {ms:.4f} ms/step, eager {eager_ms:.4f} ms/step "
        f"(fused path: {plan.fused}, {plan.n_units} units, {plan.step_threads} threads)")

    real_bytes = 8 if args.precision == "f64" else 4
    touched = touched_points_device(wl.X, wl.grid, device=dev)
    bytes_step = algorithmic_bytes(wl, touched, real_bytes)
    gbs = bytes_step / (ms * 1e-3) / 1e9
    value = wl.n_nodes / (ms * 1e-3)
    launch = {"threads": plan.step_threads, "tile_bytes": plan.tile_bytes, "units": plan.n_units}
    traffic, traffic_src = load_traffic(wl.name, args.precision, launch)
    kernel = (f"k_step_fused<{'double' if args.precision == 'f64' else 'float'}, "
              f"{plan.step_threads}, false>") if plan.fused else "unfused step"
    if plan.patched_bodies:
        kernel += " + geometry and commit passes"

    out = {
        "metric": "Lagrangian node-steps/s (forces+interp+spread+update)",
        "value": value, "unit": "node-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.precision,
        "data": "synthetic (seeded icosphere drops, random-Fourier MAC velocity)",
        "config": {"workload": wl.name, "bodies": wl.n_bodies, "nodes": wl.n_nodes,
                   "edges": wl.n_edges, "faces": wl.n_faces,
                   "grid": [wl.grid.nx, wl.grid.ny, wl.grid.nz], "dt": wl.dt,
                   "launch_options": options, "work_units": plan.n_units,
                   "threads": plan.step_threads, "timing": "hipGraph replay of the timed steps",
                   "eager_ms_per_step": eager_ms},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel,
                     "algorithmic_bytes_per_launch": bytes_step,
                     "bytes_per_node": bytes_step / wl.n_nodes,
                     "touched_grid_points": touched,
                     "traffic_source": traffic_src,
                     # what bounds the step: VALU issue (SQ counters of the same
                     # kernel, committed beside the traffic record)
                     "valu_issue": load_valu(wl.name, args.precision, launch, ms)},
    }
    if tuning is not None:
        out["autotune"] = {"choice": options, "cache": tune_info,
                           "searched": [{"options": r["options"], "ms": r["ms"],
                                         "stage": r["stage"], "units": r["units"],
                                         "threads": r["threads"]} for r in tuning]}
    del plan, X, u, f
    torch.cuda.empty_cache()

    legs = set() if args.no_extras else set(args.legs.split(","))
    if legs:
        extras = {}
    if "other" in legs:
        other = "f32" if args.precision == "f64" else "f64"
        plan2, ref2, k2, X2, u2, f2, V2, A2 = setup(other)
        ms2e = time_steps(N, plan2, X2, ref2, k2, u2, f2, wl.dt, V2, A2, args.steps,
                          args.warmup, stream, torch)
        ms2 = time_graph(N, plan2, X2, ref2, k2, u2, f2, wl.dt, V2, A2, args.steps,
                         args.warmup, torch)
        code, flags = N.ip_plan_status(plan2)
        if code != N.IP_OK:
            raise SystemExit(f"device status {code} flags {flags} in the {other} leg")
        b2 = algorithmic_bytes(wl, touched, 8 if other == "f64" else 4)
        extras[f"{other}_ms_per_step"] = ms2
        extras[f"{other}_eager_ms_per_step"] = ms2e
        extras[f"{other}_node_steps_per_s"] = wl.n_nodes / (ms2 * 1e-3)
        extras[f"{other}_roofline"] = roofline_block(
            b2, ms2, f"k_step_fused<{'double' if other == 'f64' else 'float'}, "
                     f"{plan2.step_threads}, false>", {"bytes_per_node": b2 / wl.n_nodes})
        launch2 = {"threads": plan2.step_threads, "tile_bytes": plan2.tile_bytes,
                   "units": plan2.n_units}
        traffic2, traffic2_src = load_traffic(wl.name, other, launch2)
        if traffic2 is not None:
            extras[f"{other}_roofline"].update({"traffic": traffic2,
                                                "traffic_source": traffic2_src})
        valu2 = load_valu(wl.name, other, launch2, ms2)
        if valu2 is not None:
            extras[f"{other}_roofline"]["valu_issue"] = valu2
        log(f"{other}: graph replay {ms2:.4f} ms/step, eager {ms2e:.4f} ms/step, "
            f"{extras[f'{other}_roofline']['frac']:.1%} of HBM")
        del plan2, X2, u2, f2
        torch.cuda.empty_cache()
    if "weights" in legs:
        # per-edge weights on ks and kb bound to a plan of the same shape: the
        # weighted kernel reads one more 16-byte value per edge record
        plan3, ref3, k3, X3, u3, f3, V3, A3 = setup(args.precision)
        gw = torch.Generator(device=dev)
        gw.manual_seed(1003)
        ew = 0.5 + 1.5 * torch.rand((wl.n_edges, 2), generator=gw, device=dev,
                                    dtype=torch.float64)
        N.ip_plan_bind_edge_weights(plan3, ew)
        ms3 = time_steps(N, plan3, X3, ref3, k3, u3, f3, wl.dt, V3, A3, args.steps,
                         args.warmup, stream, torch)
        code, flags = N.ip_plan_status(plan3)
        if code != N.IP_OK:
            raise SystemExit(f"device status {code} flags {flags} in the weights leg")
        extras["edge_weights_ms_per_step"] = ms3
        extras["edge_weights_over_unweighted"] = ms3 / ms
        log(f"per-edge weights bound: {ms3:.4f} ms/step ({ms3 / ms:.3f}x the unweighted step)")
        del plan3, X3, u3, f3, ew
        torch.cuda.empty_cache()
    if "backward" in legs and args.precision == "f64":
        extras.update(backward_leg(N, W, args.bodies, dev, torch, log))
    if "mls" in legs:
        extras.update(mls_leg(N, W, args.bodies, dev, torch, log))
        torch.cuda.empty_cache()
    if "uneven" in legs:
        extras.update(uneven_leg(N, W, dev, torch, log))
    if legs:
        out["extras"] = extras

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(wl, u_host, log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
