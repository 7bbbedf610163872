"""ip_forces_noalloc, the variant of ip_forces whose workspace is the
library's static device scratch: through the C-ABI, against ip_forces on the
same plan, on two calls in a row (the second on a smaller batch, so the
scratch holds the first call's larger contents), in FP64 and FP32; a plan
whose workspace exceeds the scratch is refused before any launch."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1612_03399_amd import native as N
from paper_1612_03399_amd import workload as W

from gpu_common import DEV, constants, dev, gpu_reference_from_oracle, host

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def both(wl, precision, with_va):
    """F (and V, A, W) from ip_forces and from ip_forces_noalloc on one plan."""
    ref = O.reference(wl)
    plan = N.Plan(wl, wl.grid, precision)
    gref = gpu_reference_from_oracle(ref, precision)
    k = constants(wl)
    X = dev(wl.X)
    out = []
    for fn in (N.ip_forces, N.ip_forces_noalloc):
        F = torch.full((wl.n_nodes, 3), float("nan"), dtype=plan.dtype, device=DEV)
        V = torch.full((wl.n_bodies,), float("nan"), dtype=torch.float64, device=DEV)
        A = torch.full_like(V, float("nan"))
        Wt = torch.full((wl.n_bodies, 4), float("nan"), dtype=torch.float64, device=DEV)
        if with_va:
            fn(plan, X, gref, k, F, V=V, A=A, W=Wt)
        else:
            fn(plan, X, gref, k, F, W=Wt)
        code, flags = N.ip_plan_status(plan)
        assert code == N.IP_OK, flags
        out.append((host(F), host(V), host(A), host(Wt)))
    return out


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_noalloc_matches_ip_forces_twice(precision):
    # first call: four level-3 drops; second: one level-2 drop (smaller), so
    # the scratch still holds the first call's slots beyond the second's
    cases = [(W.small_suspension(4, 3, 64, r=0.08), True),
             (W.small_suspension(1, 2, 32), False)]
    for wl, with_va in cases:
        say("noalloc", precision, wl.name, wl.n_nodes, "nodes, V/A given" if with_va else "")
        (F0, V0, A0, W0), (F1, V1, A1, W1) = both(wl, precision, with_va)
        assert np.isfinite(F0).all() and np.isfinite(W0).all()
        # the same kernels on the same inputs: the same bits
        assert np.array_equal(F1, F0)
        assert np.array_equal(W1, W0)
        if with_va:
            assert np.array_equal(V1, V0) and np.array_equal(A1, A0)
        else:                                     # V, A not requested: untouched
            assert np.isnan(V1).all() and np.isnan(A1).all()


def test_noalloc_refuses_oversized_plan():
    wl = W.suspension(n_bodies=64, level=4, r=0.02, n=64, config=13, steps=1)
    plan = N.Plan(wl, wl.grid, "f64")
    assert 3 * 8 * (4 * plan.E + 3 * plan.F) > 64 << 20
    gref = gpu_reference_from_oracle(O.reference(wl), "f64")
    F = torch.full((wl.n_nodes, 3), 7.0, dtype=torch.float64, device=DEV)
    with pytest.raises(N.IpibmError) as e:
        N.ip_forces_noalloc(plan, dev(wl.X), gref, constants(wl), F)
    assert e.value.code == N.IP_ERR_ARG and "static array" in str(e.value)
    torch.cuda.synchronize()
    assert (F == 7.0).all().item()
    # the plan stays usable, and ip_forces itself takes it
    N.ip_forces(plan, dev(wl.X), gref, constants(wl), F)
    assert N.ip_plan_status(plan)[0] == N.IP_OK
