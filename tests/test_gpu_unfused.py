"""GPU parity of the unfused step and reverse step (ip_step / ip_step_vjp on a
plan whose largest body fits one work unit but leaves too little LDS for the
grid tile: a 3068-node open sheet).  These paths run element kernels, the
gather, interpolation, spreading and the update as separate launches, and the
reverse step's constant gradients come from per-element dot products."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1612_03399_amd import native as N
from paper_1612_03399_amd import workload as W

from gpu_common import (DEV, constants, dev, gpu_reference_from_oracle, host, per_body_rel,
                        rel_inf, step_error)

pytestmark = pytest.mark.gpu


def sheet_and_drop():
    """A wavy open sheet of 51 x 58 quads (3068 nodes) beside a level-2 drop,
    on a 32^3 grid."""
    st, faces = W.flat_patch(51, 58, 0.40, 0.45)
    Xref = np.column_stack([0.25 + st[:, 0], 0.25 + st[:, 1], np.full(len(st), 0.45)])
    rng = np.random.default_rng(40)
    X = Xref.copy()
    X[:, 2] += 0.01 * np.sin(2 * np.pi * st[:, 0] / 0.4) * np.cos(2 * np.pi * st[:, 1] / 0.45)
    X += rng.normal(0, 0.0005, size=X.shape)
    v, f = W.icosphere(2)
    dref = np.array([0.45, 0.75, 0.75]) + 0.08 * v
    drop = 0.45 + (dref - 0.45) * np.array([1.1, 1.0, 0.95]) + rng.normal(0, 0.001, size=v.shape)
    bodies = [dict(X=X, Xref=Xref, faces=faces, closed=False),
              dict(X=drop, Xref=dref, faces=f, closed=True)]
    return W._assemble(bodies, "sheet_drop", W.Grid(32, 32, 32, 1.0 / 32), 1e-3, 1, "f64",
                       (1.0, 0.01, 0.1, 1.0))


def kmat(wl):
    return np.stack([wl.ks, wl.kb, wl.kA, wl.kV]).astype(np.float64)


@pytest.mark.parametrize("weighted", [False, True], ids=["plain", "edge_weights"])
def test_unfused_step_and_vjp_parity(weighted):
    wl = sheet_and_drop()
    assert wl.node_off[1] == 3068
    ref = O.reference(wl)
    ew = np.random.default_rng(2).uniform(0.5, 2.0, size=(wl.n_edges, 2)) if weighted else None
    plan = N.Plan(wl, wl.grid, "f64")
    print("unfused", weighted, "fused:", plan.fused, flush=True)
    assert not plan.fused                   # the path under test
    if weighted:
        N.ip_plan_bind_edge_weights(plan, dev(ew))
    gref = gpu_reference_from_oracle(ref, "f64")
    k = constants(wl)
    u = wl.velocity()

    # one step: X and the spread field
    f_want = np.zeros_like(u)
    want = O.step(wl, wl.X, ref, u, wl.dt, f_want, ew=ew)
    X = dev(wl.X)
    f = torch.zeros(u.shape, dtype=torch.float64, device=DEV)
    N.ip_step(plan, X, gref, k, dev(u), f, wl.dt)
    code, flags = N.ip_plan_status(plan)
    assert code == N.IP_OK, flags
    assert step_error(wl, host(X), want["X"], wl.X, 1e-12) <= 1.0
    assert rel_inf(host(f), f_want) <= 1e-12

    # reverse step: lam = lam' + dt J_U^T P + dt^2/m dF(P), gk from the
    # family forces at unit constants, gu = dt h^3 spread(P)
    dt = wl.dt
    rng = np.random.default_rng(9)
    lam1 = rng.normal(size=wl.X.shape)
    nb = O.node_body(wl)
    c2 = (dt * dt / np.asarray(wl.mass, np.float64))[nb][:, None]
    P = (1 - np.asarray(wl.pinned, np.float64))[:, None] * lam1
    J = O.interp_jac(wl.X, wl.grid, u)
    dF = O.forces_jvp(wl, wl.X, P, ref, kmat(wl), ew=ew)
    want_lam = lam1 + dt * np.einsum("lde,ld->le", J, P) + c2 * dF
    fu = O.forces(wl, wl.X, ref, np.ones((4, wl.n_bodies)), families=True, ew=ew)["Ffam"]
    want_gk = np.stack([np.bincount(nb, (fu[s] * P).sum(axis=1) * c2[:, 0],
                                    minlength=wl.n_bodies) for s in range(4)])
    want_gu = dt * wl.grid.h ** 3 * O.spread(wl.X, P, wl.grid)
    gk = torch.zeros(4, wl.n_bodies, dtype=torch.float64, device=DEV)
    gu = torch.zeros(u.shape, dtype=torch.float64, device=DEV)
    lam = N.ip_step_vjp(plan, dev(wl.X), gref, k, dev(u), dt, dev(lam1), gk=gk, gu=gu)
    code, flags = N.ip_plan_status(plan)
    assert code == N.IP_OK, flags
    e_lam = per_body_rel(host(lam) - lam1, want_lam - lam1, wl.node_off)
    e_gk = max(rel_inf(host(gk)[s], want_gk[s]) for s in range(4) if np.abs(want_gk[s]).max() > 0)
    e_gu = rel_inf(host(gu), want_gu)
    print(f"  lam {e_lam:.2e}  gk {e_gk:.2e}  gu {e_gu:.2e}", flush=True)
    assert e_lam <= 1e-12 and e_gk <= 1e-11 and e_gu <= 1e-12
