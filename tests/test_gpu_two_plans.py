"""Several live plans in one process: each plan's fused kernels need their
own dynamic LDS (it depends on the largest unit), and a plan built later must
not leave an earlier one unable to launch."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1612_03399_amd import native as N
from paper_1612_03399_amd import workload as W

from gpu_common import DEV, constants, dev, gpu_reference_from_oracle, host, step_error

pytestmark = pytest.mark.gpu


def sheet(nq):
    """One open wavy sheet of nq x nq quads ((nq + 1)^2 nodes) on 32^3."""
    st, faces = W.flat_patch(nq, nq, 0.3, 0.3)
    Xref = np.column_stack([0.35 + st[:, 0], 0.35 + st[:, 1], np.full(len(st), 0.5)])
    X = Xref.copy()
    X[:, 2] += 0.01 * np.sin(2 * np.pi * st[:, 0] / 0.3) * np.sin(2 * np.pi * st[:, 1] / 0.3)
    return W._assemble([dict(X=X, Xref=Xref, faces=faces, closed=False)], f"sheet{nq}",
                       W.Grid(32, 32, 32, 1.0 / 32), 1e-3, 1, "f64", (1.0, 0.01, 0.1, 1.0))


def test_earlier_plan_still_launches():
    # 144 nodes, then 121: the second plan's units need a few bytes less LDS
    wa, wb = sheet(11), sheet(10)
    plans = []
    for wl in (wa, wb):
        plan = N.Plan(wl, wl.grid, "f64")
        N.ip_plan_bind_reference(plan, gpu_reference_from_oracle(O.reference(wl), "f64"))
        assert plan.fused
        plans.append(plan)
    for wl, plan in ((wa, plans[0]), (wb, plans[1]), (wa, plans[0])):
        u = wl.velocity()
        want = O.step(wl, wl.X, O.reference(wl), u, wl.dt, None)
        X = dev(wl.X)
        f = torch.zeros(u.shape, dtype=torch.float64, device=DEV)
        N.ip_step(plan, X, None, constants(wl), dev(u), f, wl.dt)
        code, flags = N.ip_plan_status(plan)
        assert code == N.IP_OK, flags
        assert step_error(wl, host(X), want["X"], wl.X, 1e-12) <= 1.0


def test_plan_with_a_capped_tile_does_not_shrink_another():
    """A plan whose options cap the tile needs far less LDS than a default
    plan of the same mesh; building it second must not stop the first."""
    wl = W.small_suspension(4, 4, 128, r=0.04)
    ref = O.reference(wl)
    big = N.Plan(wl, wl.grid, "f64")
    small = N.Plan(wl, wl.grid, "f64", {"tile_bytes": 4096})
    assert big.tile_bytes > 4 * small.tile_bytes
    u = wl.velocity()
    want = O.step(wl, wl.X, ref, u, wl.dt, None)
    for plan in (big, small, big):
        N.ip_plan_bind_reference(plan, gpu_reference_from_oracle(ref, "f64"))
        X = dev(wl.X)
        f = torch.zeros(u.shape, dtype=torch.float64, device=DEV)
        N.ip_step(plan, X, None, constants(wl), dev(u), f, wl.dt)
        code, flags = N.ip_plan_status(plan)
        assert code == N.IP_OK, flags
        assert step_error(wl, host(X), want["X"], wl.X, 1e-12) <= 1.0
