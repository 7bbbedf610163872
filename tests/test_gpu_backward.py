"""GPU parity of the derivative entry points (FP64 plans) against the oracle:
the forces' directional derivative (oracle: complex step), one reverse step
with an arbitrary adjoint (oracle: interpolation Jacobian, complex-step JVP,
unit-constant family forces, spreading), the Taylor deformation and its
gradient, and a whole differentiable rollout (oracle: rollout_grad)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1612_03399_amd import autograd as AG
from paper_1612_03399_amd import native as N
from paper_1612_03399_amd import workload as W

from gpu_common import DEV, constants, dev, gpu_reference_from_oracle, host, per_body_rel, rel_inf

pytestmark = pytest.mark.gpu

# Derivatives add one differentiation to the forward arithmetic: the forces'
# derivative is a sum of terms of the size of |F| / |edge| with the same
# rounding per term as the forces themselves, so the forward bound (1e-12
# normwise per body) carries over.  Accumulated quantities (the constants'
# gradients, sums over a body's elements; the velocity gradient, atomic sums
# on the grid) are compared normwise over the array.
TOL = 1e-12

CASES = {
    "drop_L3_64": lambda: W.config0(),
    "four_L2_32": lambda: W.small_suspension(4, 2, 32),
    "uneven_small": lambda: W.config2(n_bodies=24, n=64),
    # level-4 drops of radius 1.9 h: ~55 nodes per occupied cell, so a
    # cell's nodes are spread by several work items
    "crowded_L4_32": lambda: W.small_suspension(2, 4, 32, r=0.06),
    "ventricle_small": lambda: W.config3(freq=12, leaflet_quads=10, noise_rel=0.2,
                                         cells_per_unit=64),
    # a shell split into patches by the fused reverse step
    "ventricle_patched": lambda: W.config3(freq=40, leaflet_quads=30, noise_rel=0.2,
                                           cells_per_unit=96),
    # 300 units: two full rounds of the chunked deal of units to the XCDs
    # (128 units each) and a ragged tail of 44 in plain order
    "many_L1_64": lambda: W.small_suspension(300, 1, 64, r=0.03),
}


def say(*a):
    print(*a, flush=True)


def setup(case, options=None):
    wl = CASES[case]()
    ref = O.reference(wl)
    plan = N.Plan(wl, wl.grid, "f64", options)
    return wl, ref, plan, gpu_reference_from_oracle(ref, "f64"), constants(wl)


def kmat(wl):
    return np.stack([wl.ks, wl.kb, wl.kA, wl.kV]).astype(np.float64)


@pytest.mark.parametrize("case", list(CASES))
def test_forces_jvp_parity(case):
    say("forces_jvp", case)
    wl, ref, plan, gref, k = setup(case)
    dX = np.random.default_rng(7).normal(size=wl.X.shape) * 1e-2
    want = O.forces_jvp(wl, wl.X, dX, ref, kmat(wl))
    got = host(N.ip_forces_jvp(plan, dev(wl.X), dev(dX), gref, k))
    err = per_body_rel(got, want, wl.node_off)
    say("  per-body rel", err)
    assert err <= TOL


def test_forces_jvp_symmetric():
    say("forces_jvp symmetry")
    wl, ref, plan, gref, k = setup("four_L2_32")
    rng = np.random.default_rng(8)
    a, b = rng.normal(size=wl.X.shape), rng.normal(size=wl.X.shape)
    Ja = host(N.ip_forces_jvp(plan, dev(wl.X), dev(a), gref, k))
    Jb = host(N.ip_forces_jvp(plan, dev(wl.X), dev(b), gref, k))
    lhs, rhs = (a * Jb).sum(), (Ja * b).sum()
    scale = np.sqrt((a * a).sum() * (Jb * Jb).sum())
    assert abs(lhs - rhs) <= 1e-13 * scale


@pytest.mark.parametrize("case", list(CASES))
def test_step_vjp_parity(case):
    say("step_vjp", case)
    check_step_vjp(case)


#: workgroup shapes of the fused reverse step besides the default
VJP_SHAPES = {
    "t256_small_units": {"threads": 256, "wg_per_cu": 2, "unit_nodes": 384, "patch_owned": 128},
    "t128_four_per_cu": {"threads": 128, "wg_per_cu": 4, "patch_owned": 256},
    "t128_six_per_cu": {"threads": 128, "wg_per_cu": 6, "patch_owned": 128},
}


@pytest.mark.parametrize("shape", list(VJP_SHAPES))
@pytest.mark.parametrize("case", ["uneven_small", "ventricle_patched"])
def test_step_vjp_launch_shapes(case, shape):
    say("step_vjp shape", case, shape)
    plan = check_step_vjp(case, VJP_SHAPES[shape])
    assert plan.step_threads == VJP_SHAPES[shape]["threads"]


def check_step_vjp(case, options=None):
    wl, ref, plan, gref, k = setup(case, options)
    u = wl.velocity(dtype=np.float64)
    dt = wl.dt
    rng = np.random.default_rng(9)
    lam1 = rng.normal(size=wl.X.shape)
    # oracle: lam = lam1 + dt J_U^T P + (dt^2/m) dF(P), P = M lam1
    nb = O.node_body(wl)
    mask = (1 - np.asarray(wl.pinned, np.float64))[:, None]
    c2 = (dt * dt / np.asarray(wl.mass, np.float64))[nb][:, None]
    P = mask * lam1
    J = O.interp_jac(wl.X, wl.grid, u)
    dF = O.forces_jvp(wl, wl.X, P, ref, kmat(wl))
    want_lam = lam1 + dt * np.einsum("lde,ld->le", J, P) + c2 * dF
    fu = O.forces(wl, wl.X, ref, np.ones((4, wl.n_bodies)), families=True)["Ffam"]
    B = wl.n_bodies
    want_gk = np.stack([np.bincount(nb, (fu[s] * P).sum(axis=1) * c2[:, 0], minlength=B)
                        for s in range(4)])
    want_gu = dt * wl.grid.h ** 3 * O.spread(wl.X, P, wl.grid)

    # gk and gu accumulate: seed gk with values of the contribution's size
    gk0 = rng.normal(size=(4, B)) * np.abs(want_gk).max(axis=1, keepdims=True)
    gk = dev(gk0)
    gu = torch.zeros(u.shape, dtype=torch.float64, device=DEV)
    lam = N.ip_step_vjp(plan, dev(wl.X), gref, k, dev(u), dt, dev(lam1), gk=gk, gu=gu)
    e_lam = per_body_rel(host(lam) - lam1, want_lam - lam1, wl.node_off)
    e_gk = max(rel_inf(host(gk)[s], gk0[s] + want_gk[s]) for s in range(4))
    e_gu = rel_inf(host(gu), want_gu)
    say(f"  lam {e_lam:.2e}  gk {e_gk:.2e}  gu {e_gu:.2e}")
    assert e_lam <= TOL and e_gk <= 1e-11 and e_gu <= TOL
    # the adjoint may be updated in place (same result up to summation order)
    lam_in = dev(lam1)
    N.ip_step_vjp(plan, dev(wl.X), gref, k, dev(u), dt, lam_in, lam=lam_in)
    assert per_body_rel(host(lam_in) - lam1, want_lam - lam1, wl.node_off) <= TOL
    return plan


@pytest.mark.parametrize("case", ["drop_L3_64", "four_L2_32", "uneven_small"])
def test_taylor_parity(case):
    say("taylor", case)
    wl, ref, plan, gref, k = setup(case)
    Dw, _ = O.taylor(wl, wl.X)
    D = host(AG.taylor(plan, dev(wl.X)))
    assert np.abs(D - Dw).max() <= 1e-12 * max(1.0, np.abs(Dw).max())
    Ds = Dw + 0.05
    lw, gw = O.taylor_loss_grad(wl, wl.X, Ds)
    D2, loss, gX = N.ip_taylor(plan, dev(wl.X), dev(Ds))
    assert abs(host(loss).sum() - lw) <= 1e-12 * abs(lw)
    err = per_body_rel(host(gX), gw, wl.node_off)
    say("  grad per-body rel", err)
    assert err <= 1e-10


@pytest.mark.parametrize("case", ["four_L2_32", "ventricle_small", "ventricle_patched"])
def test_rollout_gradients(case):
    """Three explicit steps, loss = sum_b (D_b - D*_b)^2 on the final
    positions, gradients with respect to X0, the constants and u."""
    say("rollout", case)
    wl, ref, plan, gref, k = setup(case)
    u = wl.velocity(dtype=np.float64) * 50.0
    dt, steps = wl.dt, 3
    Dw, _ = O.taylor(wl, wl.X)
    Ds = Dw + 0.05
    want = O.rollout_grad(wl, wl.X, ref, u, dt, steps, Ds, kmat(wl))

    X0 = dev(wl.X).requires_grad_(True)
    ut = dev(u).requires_grad_(True)
    km = dev(kmat(wl)).requires_grad_(True)
    mass = dev(np.asarray(wl.mass, np.float64))
    Xf = AG.rollout(plan, X0, ut, km, gref, mass, dt, steps)
    loss = AG.taylor_loss(plan, Xf, dev(Ds))
    loss.backward()
    e_x = per_body_rel(host(Xf), want["X_final"], wl.node_off)
    e_l = abs(loss.item() - want["loss"]) / abs(want["loss"])
    e_g = per_body_rel(host(X0.grad), want["gX0"], wl.node_off)
    e_k = max(rel_inf(host(km.grad)[s], want["gk"][s]) for s in range(4))
    e_u = rel_inf(host(ut.grad), want["gu"])
    say(f"  X {e_x:.2e} loss {e_l:.2e} gX0 {e_g:.2e} gk {e_k:.2e} gu {e_u:.2e}")
    assert e_x <= 1e-13 and e_l <= 1e-10
    # the reverse pass runs along the library's own forward trajectory, which
    # differs from the oracle's by rounding; three steps keep that below 1e-10
    assert e_g <= 1e-10 and e_k <= 1e-10 and e_u <= 1e-10


def test_derivatives_need_f64():
    say("f32 refused")
    wl = W.config0()
    plan = N.Plan(wl, wl.grid, "f32")
    ref = O.reference(wl)
    gref = gpu_reference_from_oracle(ref, "f32")
    X = dev(wl.X)
    with pytest.raises(N.IpibmError) as e:
        N.ip_forces_jvp(plan, X, X, gref, constants(wl))
    assert e.value.code == N.IP_ERR_UNSUPPORTED


@pytest.mark.parametrize("case", ["drop_L3_64", "four_L2_32", "ventricle_small"])
def test_interp_vjp_parity(case):
    """ibm_interp_vjp against the oracle: gX = J_U^T dU from the oracle's
    interpolation Jacobian, gu = h^3 spread(dU) (the transpose of
    interpolation), accumulated onto a seeded gu."""
    say("interp_vjp", case)
    wl, ref, plan, gref, k = setup(case)
    u = wl.velocity(dtype=np.float64)
    rng = np.random.default_rng(31)
    dU = rng.normal(size=wl.X.shape)
    J = O.interp_jac(wl.X, wl.grid, u)
    want_gX = np.einsum("lde,ld->le", J, dU)
    want_gu = wl.grid.h ** 3 * O.spread(wl.X, dU, wl.grid)
    gu0 = rng.normal(size=u.shape) * np.abs(want_gu).max()
    gu = dev(gu0)
    gX, _ = N.ibm_interp_vjp(plan, dev(wl.X), dev(u), dev(dU), gu=gu)
    e_x = per_body_rel(host(gX), want_gX, wl.node_off)
    e_u = rel_inf(host(gu) - gu0, want_gu)
    say(f"  gX {e_x:.2e}  gu {e_u:.2e}")
    assert e_x <= TOL and e_u <= TOL
    # the adjoint identity <dU, I(X) v> = <I^T dU, v> for a random field v
    v = rng.normal(size=u.shape)
    Iv = host(N.ibm_interp(plan, dev(wl.X), dev(v)))
    gv = torch.zeros(u.shape, dtype=torch.float64, device=DEV)
    N.ibm_interp_vjp(plan, dev(wl.X), dev(u), dev(dU), gu=gv, want_gX=False)
    lhs, rhs = (dU * Iv).sum(), (host(gv) * v).sum()
    assert abs(lhs - rhs) <= 1e-12 * np.abs(dU * Iv).sum()


def test_interp_vjp_needs_f64():
    wl = CASES["drop_L3_64"]()
    plan = N.Plan(wl, wl.grid, "f32")
    X = dev(wl.X)
    u = dev(wl.velocity(dtype=np.float64))
    with pytest.raises(N.IpibmError):
        N.ibm_interp_vjp(plan, X, u, X)
