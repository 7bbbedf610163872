"""Parity at full size: the 1000-drop suspension on 256^3 (the measured
workload, in the launch configuration the bench times: one fused step for the
whole batch), the ventricle shell with pinned leaflets on 384x384x512, and the
uneven 4096-body batch on 512^3 (sampled bodies).  The oracle is fast enough
for a whole step of the first two; for the uneven batch it steps sampled bodies
one by one and, for the grid force, every body whose support can reach theirs."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1612_03399_amd import native as N
from paper_1612_03399_amd import workload as W

from gpu_common import (DEV, TOL, constants, dev, gpu_reference_from_oracle, host,
                        oracle_reference_as_seen, rel_inf, step_error, subset)

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def gpu_step(wl, ref, u, precision, bound=True):
    """One ip_step as the bench runs it: reference bound to the plan."""
    rdt = N.real_dtype(precision)
    plan = N.Plan(wl, wl.grid, precision)
    X = dev(wl.X)
    f = torch.zeros(u.shape, dtype=rdt, device=DEV)
    V = torch.empty(wl.n_bodies, dtype=torch.float64, device=DEV)
    A = torch.empty_like(V)
    gref = gpu_reference_from_oracle(ref, precision)
    if bound:
        N.ip_plan_bind_reference(plan, gref)
        gref = None
    N.ip_step(plan, X, gref, constants(wl), dev(u, rdt), f, wl.dt, V=V, A=A)
    code, flags = N.ip_plan_status(plan)
    assert code == N.IP_OK, flags
    return plan, host(X), host(f).astype(np.float64), host(V), host(A)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_suspension_full_step(precision):
    say("full suspension", precision)
    wl = W.config1(precision=precision)
    ref = O.reference(wl)
    u = wl.velocity()
    if precision == "f32":
        u = u.astype(np.float32).astype(np.float64)
    plan, Xg, fg, Vg, Ag = gpu_step(wl, ref, u, precision)
    assert plan.fused                       # the bench's launch configuration
    say("  gpu done; oracle step ...")
    f_want = np.zeros_like(u)
    want = O.step(wl, wl.X, oracle_reference_as_seen(ref, precision), u, wl.dt, f_want)
    e_x = step_error(wl, Xg, want["X"], wl.X, TOL[precision])
    e_f = rel_inf(fg, f_want)
    e_v = np.abs(Vg / want["V"] - 1).max()
    say(f"  X {e_x:.3f} (<= 1)  f {e_f:.2e}  V {e_v:.2e}")
    assert e_x <= 1.0 and e_f <= TOL[precision] and e_v <= 1e-12


def test_ventricle_full_step():
    say("full ventricle")
    wl = W.config3(noise_rel=0.2)
    ref = O.reference(wl)
    say("  velocity ...")
    u = wl.velocity()
    plan, Xg, fg, Vg, Ag = gpu_step(wl, ref, u, "f64")
    say("  gpu done; oracle step ...")
    f_want = np.zeros_like(u)
    want = O.step(wl, wl.X, ref, u, wl.dt, f_want)
    e_x = step_error(wl, Xg, want["X"], wl.X, TOL["f64"])
    e_f = rel_inf(fg, f_want)
    say(f"  X {e_x:.3f} (<= 1)  f {e_f:.2e}")
    assert e_x <= 1.0 and e_f <= TOL["f64"]
    pin = wl.pinned == 1
    assert pin.any() and np.array_equal(Xg[pin], wl.X[pin])


def body_spheres(wl):
    c = np.empty((wl.n_bodies, 3))
    r = np.empty(wl.n_bodies)
    for b in range(wl.n_bodies):
        x = wl.X[wl.node_off[b]:wl.node_off[b + 1]]
        c[b] = x.mean(axis=0)
        r[b] = np.sqrt(((x - c[b]) ** 2).sum(axis=1).max())
    return c, r


def support_mask(X, grid):
    """Points of the three lattices within the 27-point supports of X."""
    n = np.array([grid.nx, grid.ny, grid.nz])
    m = np.zeros((3, grid.nz, grid.ny, grid.nx), bool)
    for d in range(3):
        off = np.array(W.MAC_OFFSETS[d])
        c = np.floor(X / grid.h - off + 0.5).astype(np.int64)
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    i = (c + np.array([dx, dy, dz])) % n
                    m[d, i[:, 2], i[:, 1], i[:, 0]] = True
    return m


def test_uneven_full_sampled():
    say("full uneven (sampled)")
    wl = W.config2()
    ref = O.reference(wl)
    say(f"  {wl.n_bodies} bodies, {wl.n_nodes} nodes; velocity ...")
    u = wl.velocity(dtype=np.float32).astype(np.float64)
    plan, Xg, fg, Vg, Ag = gpu_step(wl, ref, u, "f32")
    say("  gpu done; sampled oracle ...")
    rng = np.random.default_rng(17)
    levels = wl.extra["levels"]
    sample = np.concatenate([rng.choice(np.flatnonzero(levels == L), 2, replace=False)
                             for L in (2, 3, 4, 5)])
    oref = oracle_reference_as_seen(ref, "f32")
    sub = subset(wl, sample)
    want = O.step(sub, sub.X, oracle_reference_as_seen(O.reference(sub), "f32"), u, wl.dt,
                  np.zeros_like(u))
    Xg_s = np.concatenate([Xg[wl.node_off[b]:wl.node_off[b + 1]] for b in sample])
    e_x = step_error(sub, Xg_s, want["X"], sub.X, TOL["f32"])
    # grid force around the sampled bodies: every body whose support can reach
    c, r = body_spheres(wl)
    reach = r + 3.0 * wl.grid.h
    near = set()
    for b in sample:
        d = c - c[b]
        d -= np.round(d)                     # unit periodic box
        near |= set(np.flatnonzero(np.sqrt((d * d).sum(axis=1)) < reach + reach[b]).tolist())
    nsub = subset(wl, sorted(near))
    f_want = np.zeros_like(u)
    O.step(nsub, nsub.X, oracle_reference_as_seen(O.reference(nsub), "f32"), u, wl.dt, f_want)
    m = support_mask(sub.X, wl.grid)
    e_f = rel_inf(fg[m], f_want[m])
    say(f"  X {e_x:.3f} (<= 1)  f {e_f:.2e} over {m.sum()} points, {len(near)} bodies")
    assert e_x <= 1.0 and e_f <= TOL["f32"]
    del oref
