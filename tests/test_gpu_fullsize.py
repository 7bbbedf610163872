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

from gpu_common import (DEV, TOL, constants, dev, gpu_reference_from_oracle, host, near_bodies,
                        oracle_reference_as_seen, rel_inf, step_error, subset, support_mask)

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def gpu_step(wl, ref, u, precision, bound=True, options=None):
    """One ip_step as the bench runs it: reference bound to the plan."""
    rdt = N.real_dtype(precision)
    plan = N.Plan(wl, wl.grid, precision, options)
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


def uneven_sampled_check(wl, ref, u, options, per_level=16, seed=17):
    """One fused step of the whole uneven batch with the given launch options;
    the new positions of per_level sampled bodies of each level against the
    oracle stepping them alone, and the grid force on the supports of the
    sampled bodies against the oracle stepping every body whose support can
    reach theirs."""
    plan, Xg, fg, Vg, Ag = gpu_step(wl, ref, u, "f32", options=options)
    levels = wl.extra["levels"]
    rng = np.random.default_rng(seed)
    sample = np.sort(np.concatenate([rng.choice(np.flatnonzero(levels == L), per_level,
                                                replace=False) for L in (2, 3, 4, 5)]))
    sizes = np.diff(np.asarray(wl.node_off))
    say(f"  options {options}: {plan.n_units} units, {plan.patched_bodies} patched bodies; "
        f"sample of {len(sample)} bodies, {int((sizes[sample] > 3072).sum())} of them level 5")
    sub = subset(wl, sample)
    want = O.step(sub, sub.X, oracle_reference_as_seen(O.reference(sub), "f32"), u, wl.dt,
                  np.zeros_like(u))
    Xg_s = np.concatenate([Xg[wl.node_off[b]:wl.node_off[b + 1]] for b in sample])
    e_x = step_error(sub, Xg_s, want["X"], sub.X, TOL["f32"])
    # grid force around the sampled bodies: every body whose support can reach
    near = near_bodies(wl, sample)
    nsub = subset(wl, near)
    f_want = np.zeros_like(u)
    O.step(nsub, nsub.X, oracle_reference_as_seen(O.reference(nsub), "f32"), u, wl.dt, f_want)
    m = support_mask(sub.X, wl.grid)
    e_f = rel_inf(fg[m], f_want[m])
    say(f"  X {e_x:.3f} (<= 1)  f {e_f:.2e} over {m.sum()} points, {len(near)} bodies")
    assert e_x <= 1.0 and e_f <= TOL["f32"]
    return plan


@pytest.fixture(scope="module")
def uneven():
    wl = W.config2()
    ref = O.reference(wl)
    say(f"  {wl.n_bodies} bodies, {wl.n_nodes} nodes; velocity ...")
    u = wl.velocity(dtype=np.float32).astype(np.float64)
    return wl, ref, u


#: the default split, and the shape the autotuner picks on this batch (two
#: 384-thread workgroups per compute unit, most cell boxes in LDS tiles, the
#: others spread and interpolated directly against the grid)
UNEVEN_SHAPES = {"default": None, "t384_two_per_cu": {"threads": 384, "wg_per_cu": 2},
                 "t128_four_per_cu": {"threads": 128, "wg_per_cu": 4, "patch_owned": 256},
                 "t128_six_per_cu": {"threads": 128, "wg_per_cu": 6, "patch_owned": 128}}


@pytest.mark.parametrize("shape", list(UNEVEN_SHAPES))
def test_uneven_full_sampled(uneven, shape):
    say("full uneven (sampled)", shape)
    wl, ref, u = uneven
    plan = uneven_sampled_check(wl, ref, u, UNEVEN_SHAPES[shape])
    assert plan.patched_bodies > 0      # the level-5 bodies run as patches


def test_rollout_gradient_full_size():
    """Differentiation at full size: the 1000-drop suspension, 10 steps, loss
    sum_b (D_b - D*_b)^2, gradients by the library's reverse rollout.

    (1) Against the oracle's analytic gradient, drop by drop on a sample: each
    drop's loss depends on its own nodes and constants only (the velocity field
    is given), so the oracle's rollout of a drop alone gives that drop's rows of
    dL/dX0 and its column of dL/dk.  The sample includes drop 22, whose
    initial jitter leaves one triangle at 0.16% of its reference area.

    (2) Against central differences of the library's own forward rollouts along
    a random direction, drop by drop (all drops perturbed at once; the
    per-drop losses separate).  At this jitter (sigma = 0.02 r, about a third
    of an edge) some triangles are nearly collapsed and the explicit update is
    stiff there, so the loss is smooth but strongly curved: measured with the
    oracle on 300 of these drops, the per-drop relative error of a central
    difference is 1.2e-6 (median) and 3.7e-5 (90th percentile) at h = 1e-6,
    1.3e-8 and 4.8e-7 at h = 1e-7, with a few stiff drops at 1e-2 either way.
    The check asserts those orders of magnitude and the second-order
    convergence between the two steps, which a wrong gradient term breaks."""
    say("full-size rollout gradient")
    from paper_1612_03399_amd import autograd as AG
    wl = W.config4()
    steps = wl.steps
    uh = wl.velocity()
    u = dev(uh)
    plan = N.Plan(wl, wl.grid, "f64")
    N.ip_plan_bind_reference(plan, N.ip_reference_from(plan, dev(wl.Xref)))
    kh = np.stack([wl.ks, wl.kb, wl.kA, wl.kV]).astype(np.float64)
    km = dev(kh).requires_grad_(True)
    mass = dev(np.asarray(wl.mass, np.float64))
    Ds = dev(wl.targets)
    X0 = dev(wl.X).requires_grad_(True)
    loss = AG.taylor_loss(plan, AG.rollout(plan, X0, u, km, None, mass, wl.dt, steps), Ds)
    loss.backward()
    code, flags = N.ip_plan_status(plan)
    assert code == N.IP_OK, flags
    gX, gk = host(X0.grad), host(km.grad)
    no = np.asarray(wl.node_off)

    # (1) sampled drops against the oracle
    sample = [22, 0, 5, 179, 333, 500, 768, 999]
    worst_x = worst_k = 0.0
    for b in sample:
        sub = subset(wl, [b])
        want = O.rollout_grad(sub, sub.X, O.reference(sub), uh, wl.dt, steps,
                              wl.targets[[b]], kh[:, [b]])
        ex = rel_inf(gX[no[b]:no[b + 1]], want["gX0"])
        ek = np.abs(gk[:, b] - want["gk"][:, 0]).max() / np.abs(want["gk"]).max()
        worst_x, worst_k = max(worst_x, ex), max(worst_k, ek)
    say(f"  oracle, {len(sample)} drops: dX0 {worst_x:.2e}  dk {worst_k:.2e}")
    assert worst_x <= 1e-8 and worst_k <= 1e-8

    # (2) per-drop central differences
    v = dev(np.random.default_rng(11).normal(size=wl.X.shape))
    an = np.bincount(np.repeat(np.arange(wl.n_bodies), np.diff(no)),
                     host(X0.grad * v).sum(axis=1), minlength=wl.n_bodies)
    Dsh = wl.targets

    def per_drop_loss(x):
        with torch.no_grad():
            Xf = AG.rollout(plan, x, u, km.detach(), None, mass, wl.dt, steps)
            return (host(AG.taylor(plan, Xf)) - Dsh) ** 2

    err = {}
    for h in (1e-6, 1e-7):
        fd = (per_drop_loss(X0.detach() + h * v) - per_drop_loss(X0.detach() - h * v)) / (2 * h)
        err[h] = np.abs(fd - an) / np.abs(an)
        q = np.quantile(err[h], [0.5, 0.9, 1.0])
        say(f"  h={h:.0e}: per-drop relative error median {q[0]:.1e} p90 {q[1]:.1e} max {q[2]:.1e}")
    assert np.median(err[1e-6]) <= 1e-5 and np.quantile(err[1e-6], 0.9) <= 1e-3
    assert np.median(err[1e-7]) <= 1e-7 and np.quantile(err[1e-7], 0.9) <= 1e-5
    # second order: ten times smaller a step, about a hundred times smaller an error
    assert np.median(err[1e-7]) <= 0.05 * np.median(err[1e-6])
