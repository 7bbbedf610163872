"""Repeatability of the paths that add with atomics (the fused step's LDS
accumulators and grid flush, MLS spreading), and the status word for a
non-finite position: the kernels map a non-finite coordinate to a lattice
cell inside the grid (so every access stays in bounds), the values it touches
become non-finite, and the step reports IP_STATUS_NONFINITE."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1612_03399_amd import native as N
from paper_1612_03399_amd import workload as W

from gpu_common import DEV, constants, dev, gpu_reference_from_oracle, host, rel_inf

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def one_step(plan, wl, X0, k, u):
    X = dev(X0)
    f = torch.zeros(u.shape, dtype=torch.float64, device=DEV)
    N.ip_step(plan, X, None, k, u, f, wl.dt)
    return host(X), host(f)


def body_rel(dA, dB, node_off):
    """max over bodies of |dA - dB|_inf / |dB|_inf (rows = nodes)."""
    worst = 0.0
    for b in range(len(node_off) - 1):
        s = slice(node_off[b], node_off[b + 1])
        worst = max(worst, np.abs(dA[s] - dB[s]).max() / np.abs(dB[s]).max())
    return worst


@pytest.mark.parametrize("case", ["four_L4_128", "ventricle_patched"])
def test_step_repeatable(case):
    """The same step twice: the displacement agrees to the rounding of its
    summation order (the LDS accumulators and the grid flush add in a
    run-dependent order), the spread field likewise."""
    say("repeatable", case)
    wl = (W.small_suspension(4, 4, 128, r=0.04) if case == "four_L4_128"
          else W.config3(freq=40, leaflet_quads=30, noise_rel=0.2, cells_per_unit=96))
    plan = N.Plan(wl, wl.grid, "f64")
    N.ip_plan_bind_reference(plan, gpu_reference_from_oracle(O.reference(wl), "f64"))
    k = constants(wl)
    u = dev(wl.velocity())
    X1, f1 = one_step(plan, wl, wl.X, k, u)
    X2, f2 = one_step(plan, wl, wl.X, k, u)
    e_x = body_rel(X1 - wl.X, X2 - wl.X, wl.node_off)
    e_f = rel_inf(f1, f2)
    say(f"  dX {e_x:.1e}  f {e_f:.1e}")
    # a few ulps of the largest terms of each sum, relative to the sum; the
    # field carries the run-dependent rounding of both the nodes' force sums
    # (elements added in LDS in any order; at a node where they nearly
    # cancel, a large relative change of a small force) and the grid
    # additions, so it is held normwise over the field
    assert e_x <= 1e-13 and e_f <= 1e-13
    # the pieces computed without atomics are bitwise repeatable
    U1 = host(N.ibm_interp(plan, dev(wl.X), u))
    U2 = host(N.ibm_interp(plan, dev(wl.X), u))
    assert np.array_equal(U1, U2)


def test_mls_spreading_repeatable():
    wl = W.small_suspension(4, 4, 128, r=0.04)
    plan = N.Plan(wl, wl.grid, "f64")
    Fm = dev(np.random.default_rng(4).normal(size=(wl.n_faces, 3)))
    X = dev(wl.X)
    out = []
    for _ in range(2):
        f = torch.zeros(3, wl.grid.nz, wl.grid.ny, wl.grid.nx, dtype=torch.float64, device=DEV)
        N.ibm_spread_mls(plan, X, Fm, 0.4, f)
        out.append(host(f))
    assert rel_inf(out[0], out[1]) <= 1e-14


def test_nonfinite_position_sets_status():
    """One NaN coordinate in body 1: the step reports IP_STATUS_NONFINITE,
    the other bodies (own units; the velocity field is an input) still take
    the correct step."""
    say("nonfinite")
    wl = W.small_suspension(4, 2, 32)
    plan = N.Plan(wl, wl.grid, "f64")
    N.ip_plan_bind_reference(plan, gpu_reference_from_oracle(O.reference(wl), "f64"))
    k = constants(wl)
    u = dev(wl.velocity())
    Xc, _ = one_step(plan, wl, wl.X, k, u)
    code, flags = N.ip_plan_status(plan)
    assert code == N.IP_OK, flags
    Xbad = wl.X.copy()
    n1 = int(wl.node_off[1])
    Xbad[n1 + 3, 1] = np.nan
    Xn, _ = one_step(plan, wl, Xbad, k, u)
    code, flags = N.ip_plan_status(plan)
    assert flags & N.IP_STATUS_NONFINITE and code != N.IP_OK
    for b in (0, 2, 3):
        s = slice(int(wl.node_off[b]), int(wl.node_off[b + 1]))
        assert np.isfinite(Xn[s]).all()
        assert np.abs((Xn[s] - wl.X[s]) - (Xc[s] - wl.X[s])).max() <= \
            1e-12 * np.abs(Xc[s] - wl.X[s]).max()
    code, flags = N.ip_plan_status(plan)      # cleared by the read
    assert code == N.IP_OK and flags == 0
