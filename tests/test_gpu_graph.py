"""hipGraph capture of the fused step: replays (with eager work and
synchronisations between them) must give what the same steps give eagerly, up
to the run-dependent summation order of the LDS accumulation."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1612_03399_amd import native as N
from paper_1612_03399_amd import workload as W

from gpu_common import DEV, constants, dev, gpu_reference_from_oracle, host, rel_inf, step_error

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("case", ["four_L4_128", "uneven_small"])
def test_graph_replays_match_eager(case):
    say("graph", case)
    wl = (W.small_suspension(4, 4, 128, r=0.04) if case == "four_L4_128"
          else W.config2(n_bodies=24, n=64))
    ref = O.reference(wl)
    plan = N.Plan(wl, wl.grid, "f64")
    N.ip_plan_bind_reference(plan, gpu_reference_from_oracle(ref, "f64"))
    k = constants(wl)
    u = dev(wl.velocity())
    steps = 3

    def eager(X0):
        X = X0.clone()
        f = torch.zeros_like(u)
        for _ in range(steps):
            N.ip_step(plan, X, None, k, u, f, wl.dt)
        torch.cuda.synchronize()
        return host(X), host(f)

    X0 = dev(wl.X)
    Xe, fe = eager(X0)
    # capture the same steps on a side stream
    Xg = X0.clone()
    fg = torch.zeros_like(u)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for _ in range(steps):
            N.ip_step(plan, Xg, None, k, u, fg, wl.dt, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    for rep in range(3):
        Xg.copy_(X0)
        fg.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        e_x = step_error(wl, host(Xg), Xe, wl.X, 1e-12)
        e_f = rel_inf(host(fg), fe)
        say(f"  replay {rep}: X {e_x:.3f} (<= 1)  f {e_f:.2e}")
        assert e_x <= 1.0 and e_f <= 1e-12
        # eager work between replays
        Xe2, _ = eager(X0)
        assert step_error(wl, Xe2, Xe, wl.X, 1e-12) <= 1.0
    code, flags = N.ip_plan_status(plan)
    assert code == N.IP_OK, flags


@pytest.mark.parametrize("case", ["four_L4_128", "ventricle_patched"])
def test_graph_replays_of_the_centroid_transfers(case):
    """MLS interpolation, one-pass direct forcing and probe loads captured
    together: every replay gives the eager results (spreading to rounding)."""
    say("graph mls", case)
    wl = (W.small_suspension(4, 4, 128, r=0.04) if case == "four_L4_128"
          else W.config3(freq=40, leaflet_quads=30, noise_rel=0.2, cells_per_unit=96))
    plan = N.Plan(wl, wl.grid, "f64")
    rng = np.random.default_rng(8)
    X = dev(wl.X)
    u = dev(wl.velocity())
    p = dev(rng.normal(size=(wl.grid.nz, wl.grid.ny, wl.grid.nx)))
    Vb = dev(rng.normal(scale=0.1, size=(wl.n_faces, 3)))
    acc = dev(rng.normal(size=(wl.n_faces, 3)))
    alpha, dt, mu = 0.4, 1e-3, 0.02
    F = wl.n_faces

    def run(U, Fm, f, Fext, stream=None):
        N.ibm_interp_mls(plan, X, u, alpha, U, stream=stream)
        N.ibm_direct_forcing_mls(plan, X, Vb, u, alpha, dt, f, Fm=Fm, stream=stream)
        N.ibm_probe_loads(plan, X, u, p, alpha, mu, acc=acc, Fext=Fext, stream=stream)

    bufs = lambda: (torch.empty(F, 3, dtype=torch.float64, device=DEV),
                    torch.empty(F, 3, dtype=torch.float64, device=DEV),
                    torch.zeros_like(u), torch.empty(F, 3, dtype=torch.float64, device=DEV))
    Ue, Fme, fe, Fxe = bufs()
    run(Ue, Fme, fe, Fxe)
    torch.cuda.synchronize()
    Ue, Fme, fe, Fxe = host(Ue), host(Fme), host(fe), host(Fxe)
    Ug, Fmg, fg, Fxg = bufs()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        run(Ug, Fmg, fg, Fxg, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    for rep in range(3):
        for t in (Ug, Fmg, Fxg):
            t.fill_(7.0)
        fg.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(Ug), Ue) and np.array_equal(host(Fmg), Fme)
        assert np.array_equal(host(Fxg), Fxe)
        e_f = rel_inf(host(fg), fe)
        say(f"  replay {rep}: U, Fm, Fext identical, f {e_f:.2e}")
        assert e_f <= 1e-12
        # eager work between replays
        a, b, c, d = bufs()
        run(a, b, c, d)
        torch.cuda.synchronize()
        assert np.array_equal(host(a), Ue)
    code, flags = N.ip_plan_status(plan)
    assert code == N.IP_OK, flags
