"""Argument errors at the C-ABI with a valid plan: NULL and misaligned arrays
are rejected synchronously with IP_ERR_ARG, before any launch, and the plan
stays usable.  The misaligned views lie inside padded allocations."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle as O
from paper_1612_03399_amd import native as N
from paper_1612_03399_amd import workload as W

from gpu_common import DEV, constants, dev, gpu_reference_from_oracle, host

pytestmark = pytest.mark.gpu


def padded(shape, dtype=torch.float64):
    """A tensor of `shape` plus one spare element, and the address 4 bytes
    into it (misaligned for 8-byte values, still inside the allocation)."""
    n = int(np.prod(shape))
    t = torch.zeros(n + 1, dtype=dtype, device=DEV)
    return t, t.data_ptr() + 4


def test_null_and_misaligned_arrays_rejected():
    wl = W.config0()
    ref = O.reference(wl)
    plan = N.Plan(wl, wl.grid, "f64")
    gref = gpu_reference_from_oracle(ref, "f64")
    k = constants(wl)
    rs, ks = gref.struct(), k.struct()
    L = N.LIB
    h = plan.handle
    X = dev(wl.X)
    u = dev(wl.velocity())
    Nn, F = wl.n_nodes, wl.n_faces
    buf3N, bad3N = padded((Nn, 3))
    bufF, badF = padded((F, 3))
    bufu, badu = padded(u.shape)
    out3N = torch.zeros(Nn, 3, dtype=torch.float64, device=DEV)
    outF = torch.zeros(F, 3, dtype=torch.float64, device=DEV)
    f = torch.zeros_like(u)
    p = torch.zeros(u.shape[1:], dtype=torch.float64, device=DEV)
    xp, up, fp = X.data_ptr(), u.data_ptr(), f.data_ptr()
    calls = {
        "ip_forces X": lambda: L.ip_forces(h, bad3N, C.byref(rs), C.byref(ks), out3N.data_ptr(),
                                           None, None, None, None),
        "ip_forces F": lambda: L.ip_forces(h, xp, C.byref(rs), C.byref(ks), None, None, None,
                                           None, None),
        "ibm_interp u": lambda: L.ibm_interp(h, xp, badu, out3N.data_ptr(), None),
        "ibm_spread F": lambda: L.ibm_spread(h, xp, bad3N, fp, None),
        "ip_step f": lambda: L.ip_step(h, xp, C.byref(rs), C.byref(ks), up, badu, 1e-4, None,
                                       None, None),
        "ip_step X": lambda: L.ip_step(h, None, C.byref(rs), C.byref(ks), up, fp, 1e-4, None,
                                       None, None),
        "ibm_interp_mls U": lambda: L.ibm_interp_mls(h, xp, up, 0.4, badF, None),
        "ibm_spread_mls Fm": lambda: L.ibm_spread_mls(h, xp, None, 0.4, fp, None),
        "ibm_probe_loads p": lambda: L.ibm_probe_loads(h, xp, up, badu, None, 0.4, 0.01,
                                                       outF.data_ptr(), None),
        "ibm_probe_loads acc": lambda: L.ibm_probe_loads(h, xp, up, p.data_ptr(), badF, 0.4,
                                                         0.01, outF.data_ptr(), None),
        "ibm_interp_vjp dU": lambda: L.ibm_interp_vjp(h, xp, up, bad3N, out3N.data_ptr(), None,
                                                      None),
        "ip_centroid_to_nodes Fc": lambda: L.ip_centroid_to_nodes(h, badF, out3N.data_ptr(),
                                                                  None),
        "ip_plan_bind_edge_weights": lambda: L.ip_plan_bind_edge_weights(h, bad3N, None),
    }
    for name, call in calls.items():
        code = call()
        print(name, code, flush=True)
        assert code == N.IP_ERR_ARG, (name, code, L.ip_last_error())
    torch.cuda.synchronize()
    # nothing was written and the plan still works
    assert not out3N.any() and not outF.any() and not f.any()
    code, flags = N.ip_plan_status(plan)
    assert code == N.IP_OK and flags == 0
    Fgood = host(N.ip_forces(plan, X, gref, k))
    assert np.abs(Fgood - O.forces(wl, wl.X, ref)["F"]).max() <= 1e-12 * np.abs(Fgood).max()
    del buf3N, bufF, bufu
