"""GPU parity of the MLS transfer at the triangle centroids (ibm_interp_mls,
ibm_spread_mls) and of the centroid-to-vertex transfer (ip_centroid_to_nodes)
against the FP64 oracle, through the C-ABI: small cases element by element,
the 1000-drop batch on sampled markers and by force conservation."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1612_03399_amd import native as N
from paper_1612_03399_amd import workload as W

from gpu_common import DEV, TOL, dev, host, rel_inf

pytestmark = pytest.mark.gpu

CASES = {
    "drop_L3_64": lambda: W.config0(),
    "four_L4_128": lambda: W.small_suspension(4, 4, 128, r=0.04),
    "uneven_small": lambda: W.config2(n_bodies=24, n=64),
    "ventricle_small": lambda: W.config3(freq=12, leaflet_quads=10, noise_rel=0.2,
                                         cells_per_unit=64),
    # a shell split into patches: each face is spread by the unit owning its
    # first corner
    "ventricle_patched": lambda: W.config3(freq=40, leaflet_quads=30, noise_rel=0.2,
                                           cells_per_unit=96),
}


def say(*a):
    print(*a, flush=True)


def inputs(wl, precision, seed=5):
    rng = np.random.default_rng(seed)
    u = wl.velocity()
    Fm = rng.normal(size=(wl.n_faces, 3))
    if precision == "f32":       # the oracle sees the values the library reads
        u = u.astype(np.float32).astype(np.float64)
        Fm = Fm.astype(np.float32).astype(np.float64)
    return u, Fm


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("alpha", [0.3, 0.8])
@pytest.mark.parametrize("case", list(CASES))
def test_mls_interp_spread_parity(case, alpha, precision):
    say("mls", case, alpha, precision)
    wl = CASES[case]()
    rdt = N.real_dtype(precision)
    u, Fm = inputs(wl, precision)
    Cc, Af = O.centroids(wl, wl.X)
    U_want = O.interp_mls(Cc, wl.grid, u, alpha)
    f_want = O.spread_mls(Cc, Af, Fm, wl.grid, alpha)
    plan = N.Plan(wl, wl.grid, precision)
    X = dev(wl.X)
    U = host(N.ibm_interp_mls(plan, X, dev(u, rdt), alpha)).astype(np.float64)
    f = torch.zeros(u.shape, dtype=rdt, device=DEV)
    N.ibm_spread_mls(plan, X, dev(Fm, rdt), alpha, f)
    code, flags = N.ip_plan_status(plan)
    assert code == N.IP_OK, flags
    e_u = rel_inf(U, U_want)
    e_f = rel_inf(host(f).astype(np.float64), f_want)
    say(f"  U {e_u:.2e}  f {e_f:.2e}")
    assert e_u <= TOL[precision] and e_f <= TOL[precision]


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_centroid_to_nodes_parity(precision):
    wl = CASES["four_L4_128"]()
    rdt = N.real_dtype(precision)
    Fc = np.random.default_rng(3).normal(size=(wl.n_faces, 3))
    if precision == "f32":
        Fc = Fc.astype(np.float32).astype(np.float64)
    want = O.centroid_to_nodes(wl, Fc)
    plan = N.Plan(wl, wl.grid, precision)
    got = host(N.ip_centroid_to_nodes(plan, dev(Fc, rdt))).astype(np.float64)
    assert rel_inf(got, want) <= TOL[precision]
    # a gather: the same call gives the same bits
    again = host(N.ip_centroid_to_nodes(plan, dev(Fc, rdt))).astype(np.float64)
    assert np.array_equal(got, again)


def test_mls_rejects_bad_alpha():
    wl = CASES["drop_L3_64"]()
    plan = N.Plan(wl, wl.grid, "f64")
    X = dev(wl.X)
    u = dev(wl.velocity())
    for alpha in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(N.IpibmError):
            N.ibm_interp_mls(plan, X, u, alpha)


def test_mls_full_size_sampled():
    """The 1000-drop batch (5.12 M markers on 256^3): interpolation on 4000
    sampled markers against the oracle, and spreading by its conservation
    law sum_k f_d[k] h^3 = sum_l A_l h F_{l,d} over the whole batch."""
    say("mls full size")
    wl = W.config1()
    alpha = 0.4
    u = wl.velocity()
    plan = N.Plan(wl, wl.grid, "f64")
    X = dev(wl.X)
    U = host(N.ibm_interp_mls(plan, X, dev(u), alpha))
    Cc, Af = O.centroids(wl, wl.X)
    pick = np.random.default_rng(9).choice(wl.n_faces, 4000, replace=False)
    e_u = rel_inf(U[pick], O.interp_mls(Cc[pick], wl.grid, u, alpha))
    Fm = np.random.default_rng(10).normal(size=(wl.n_faces, 3))
    f = torch.zeros(u.shape, dtype=torch.float64, device=DEV)
    N.ibm_spread_mls(plan, X, dev(Fm), alpha, f)
    code, flags = N.ip_plan_status(plan)
    assert code == N.IP_OK, flags
    h = wl.grid.h
    tot = host(f.sum(dim=(1, 2, 3))) * h ** 3
    want = ((Af * h)[:, None] * Fm).sum(axis=0)
    scale = np.abs((Af * h)[:, None] * Fm).sum(axis=0)
    e_c = np.abs(tot - want).max() / scale.max()
    say(f"  U sampled {e_u:.2e}  conservation {e_c:.2e}")
    assert e_u <= TOL["f64"] and e_c <= 1e-12
