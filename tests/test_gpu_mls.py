"""GPU parity of the MLS transfer at the triangle centroids (ibm_interp_mls,
ibm_spread_mls, ibm_direct_forcing_mls), of the centroid-to-vertex transfer
(ip_centroid_to_nodes) and of the probe loads (ibm_probe_loads)
against the FP64 oracle, through the C-ABI: small cases element by element,
the 1000-drop batch on sampled markers and by force conservation."""
import types

import numpy as np
import pytest
import torch

import oracle as O
from paper_1612_03399_amd import native as N
from paper_1612_03399_amd import workload as W

from gpu_common import DEV, TOL, dev, host, near_bodies, rel_inf, subset, support_mask
from test_gpu_unfused import sheet_and_drop

pytestmark = pytest.mark.gpu


def wrapped_drops():
    """Two level-2 drops on a 32^3 grid: one centred on a corner of the
    periodic box (its supports wrap on every axis), one more than a box length
    outside the box on every axis (its cells wrap from beyond the grid)."""
    v, f = W.icosphere(2)
    rng = np.random.default_rng(41)
    bodies = []
    for c in ([0.0, 0.0, 0.0], [1.6, -1.3, 2.3]):
        Xref = np.array(c) + 0.08 * v
        X = Xref + rng.normal(0, 0.001, size=v.shape)
        bodies.append(dict(X=X, Xref=Xref, faces=f, closed=True))
    return W._assemble(bodies, "wrapped_drops", W.Grid(32, 32, 32, 1.0 / 32), 1e-3, 1, "f64",
                       (1.0, 0.01, 0.1, 1.0))

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
    # a plan without fused work units: spreading and direct forcing take the
    # per-marker kernels with device atomics
    "unfused_sheet_drop": sheet_and_drop,
    "wrapped_drops": wrapped_drops,
    # the staged velocity of the interpolation fits one lattice at a time
    # (a box of about 21^3 points beside 2562 positions)
    "drop_L4_box_one_lattice": lambda: W.small_suspension(1, 4, 128, r=0.0625),
    # a box larger than any tile: interpolation gathers from u, spreading
    # adds to f directly
    "drop_L4_box_too_big": lambda: W.small_suspension(1, 4, 128, r=0.3),
    # 300 units: two full rounds of the chunked deal of units to the XCDs
    # (128 units each) and a ragged tail of 44 in plain order
    "many_L1_64": lambda: W.small_suspension(300, 1, 64, r=0.03),
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
    """The 1000-drop batch (5.12 M markers on 256^3), in the launch
    configuration of the step: interpolation on 4000 sampled markers against
    the oracle; spreading of every marker's force compared point by point on
    the supports of 12 sampled drops against the oracle spreading the markers
    of every drop whose support can reach them; and the conservation law
    sum_k f_d[k] h^3 = sum_l A_l h F_{l,d} over the whole batch."""
    say("mls full size")
    wl = W.config1()
    alpha = 0.4
    u = wl.velocity()
    plan = N.Plan(wl, wl.grid, "f64")
    assert plan.fused
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
    fg = host(f)
    h = wl.grid.h
    tot = fg.sum(axis=(1, 2, 3)) * h ** 3
    want = ((Af * h)[:, None] * Fm).sum(axis=0)
    scale = np.abs((Af * h)[:, None] * Fm).sum(axis=0)
    e_c = np.abs(tot - want).max() / scale.max()
    # point by point on the supports of sampled drops
    sample = np.sort(np.random.default_rng(21).choice(wl.n_bodies, 12, replace=False))
    near = near_bodies(wl, sample)
    fo = np.asarray(wl.face_off)
    sel = np.concatenate([np.arange(fo[b], fo[b + 1]) for b in near])
    f_want = O.spread_mls(Cc[sel], Af[sel], Fm[sel], wl.grid, alpha)
    m = support_mask(Cc[np.concatenate([np.arange(fo[b], fo[b + 1]) for b in sample])], wl.grid)
    e_f = rel_inf(fg[m], f_want[m])
    say(f"  U sampled {e_u:.2e}  f {e_f:.2e} over {m.sum()} points ({len(near)} drops)  "
        f"conservation {e_c:.2e}")
    assert e_u <= TOL["f64"] and e_f <= TOL["f64"] and e_c <= 1e-12


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", list(CASES))
def test_direct_forcing_parity(case, precision):
    """ibm_direct_forcing_mls against the oracle: the marker forces
    (Vb - U)/dt and the spread field, in one pass on the GPU."""
    say("direct forcing", case, precision)
    wl = CASES[case]()
    rdt = N.real_dtype(precision)
    rng = np.random.default_rng(12)
    u, _ = inputs(wl, precision)
    Vb = rng.normal(scale=0.1, size=(wl.n_faces, 3))
    if precision == "f32":
        Vb = Vb.astype(np.float32).astype(np.float64)
    alpha, dt = 0.4, 1e-3
    Cc, Af = O.centroids(wl, wl.X)
    Fm_want, f_want = O.direct_forcing_mls(Cc, Af, Vb, wl.grid, u, alpha, dt)
    plan = N.Plan(wl, wl.grid, precision)
    X = dev(wl.X)
    f = torch.zeros(u.shape, dtype=rdt, device=DEV)
    Fm, _ = N.ibm_direct_forcing_mls(plan, X, dev(Vb, rdt), dev(u, rdt), alpha, dt, f)
    f2 = torch.zeros_like(f)
    none, _ = N.ibm_direct_forcing_mls(plan, X, dev(Vb, rdt), dev(u, rdt), alpha, dt, f2, Fm=False)
    code, flags = N.ip_plan_status(plan)
    assert code == N.IP_OK, flags
    assert none is None
    e_m = rel_inf(host(Fm).astype(np.float64), Fm_want)
    e_f = rel_inf(host(f).astype(np.float64), f_want)
    e_f2 = rel_inf(host(f2).astype(np.float64), f_want)
    say(f"  Fm {e_m:.2e}  f {e_f:.2e}  f (no Fm) {e_f2:.2e}")
    # F = (Vb - U)/dt: the rounding of U relative to |U| is amplified by
    # |U| / |Vb - U| at most, which the tolerance on Fm allows for
    amp = max(1.0, np.abs(u).max() / np.abs(Vb - 0).max())
    assert e_m <= TOL[precision] * amp and e_f <= TOL[precision] * amp and e_f2 <= TOL[precision] * amp


def test_direct_forcing_rejects_bad_dt():
    wl = CASES["drop_L3_64"]()
    plan = N.Plan(wl, wl.grid, "f64")
    X = dev(wl.X)
    u = dev(wl.velocity())
    Vb = torch.zeros(wl.n_faces, 3, dtype=torch.float64, device=DEV)
    f = torch.zeros_like(u)
    for dt in (0.0, -1e-3, float("nan")):
        with pytest.raises(N.IpibmError):
            N.ibm_direct_forcing_mls(plan, X, Vb, u, 0.4, dt, f)


def probe_inputs(wl, precision, seed=21):
    rng = np.random.default_rng(seed)
    u = wl.velocity() + rng.normal(scale=0.05, size=(3, wl.grid.nz, wl.grid.ny, wl.grid.nx))
    p = rng.normal(size=(wl.grid.nz, wl.grid.ny, wl.grid.nx))
    acc = rng.normal(size=(wl.n_faces, 3))
    if precision == "f32":
        u, p, acc = (a.astype(np.float32).astype(np.float64) for a in (u, p, acc))
    return u, p, acc


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", list(CASES))
def test_probe_loads_parity(case, precision):
    """ibm_probe_loads against the oracle on closed drops and on the open
    leaflets of the ventricle (two probes per face), with and without the
    acceleration term."""
    say("probe loads", case, precision)
    wl = CASES[case]()
    rdt = N.real_dtype(precision)
    u, p, acc = probe_inputs(wl, precision)
    alpha, mu = 0.4, 0.02
    plan = N.Plan(wl, wl.grid, precision)
    X = dev(wl.X)
    for a in (acc, None):
        want = O.probe_loads(wl, wl.X, wl.grid, u, p, alpha, mu, acc=a)
        got = N.ibm_probe_loads(plan, X, dev(u, rdt), dev(p, rdt), alpha, mu,
                                acc=None if a is None else dev(a, rdt))
        code, flags = N.ip_plan_status(plan)
        assert code == N.IP_OK, flags
        e = rel_inf(host(got).astype(np.float64), want)
        say(f"  acc {'yes' if a is not None else 'no'}: {e:.2e}")
        assert e <= TOL[precision]


def test_probe_loads_full_size_sampled():
    """The 1000-drop batch: loads on 4000 sampled faces against the oracle
    (run on those faces alone), in the launch the bench times."""
    say("probe loads full size")
    wl = W.config1()
    u, p, acc = probe_inputs(wl, "f64")
    plan = N.Plan(wl, wl.grid, "f64")
    got = host(N.ibm_probe_loads(plan, dev(wl.X), dev(u), dev(p), 0.4, 1e-3, acc=dev(acc)))
    code, flags = N.ip_plan_status(plan)
    assert code == N.IP_OK, flags
    pick = np.sort(np.random.default_rng(4).choice(wl.n_faces, 4000, replace=False))
    sub = types.SimpleNamespace(faces=np.asarray(wl.faces)[pick], closed=[1],
                                face_off=[0, pick.size])
    want = O.probe_loads(sub, wl.X, wl.grid, u, p, 0.4, 1e-3, acc=acc[pick])
    e = rel_inf(got[pick], want)
    say(f"  sampled {e:.2e}")
    assert e <= TOL["f64"]


def test_probe_loads_rejects_bad_arguments():
    wl = CASES["drop_L3_64"]()
    plan = N.Plan(wl, wl.grid, "f64")
    X = dev(wl.X)
    u = dev(wl.velocity())
    p = torch.zeros(u.shape[1:], dtype=torch.float64, device=DEV)
    for alpha, mu in ((0.0, 0.1), (float("nan"), 0.1), (0.4, -1.0), (0.4, float("inf"))):
        with pytest.raises(N.IpibmError):
            N.ibm_probe_loads(plan, X, u, p, alpha, mu)


def test_probe_loads_degenerate_face_and_empty_batch():
    """A collapsed face gets no load and sets the degenerate flag, the other
    faces match the oracle; an empty batch is a no-op."""
    wl = CASES["drop_L3_64"]()
    X = wl.X.copy()
    a, b, c = wl.faces[11]
    X[c] = X[a]
    u, p, acc = probe_inputs(wl, "f64")
    plan = N.Plan(wl, wl.grid, "f64")
    got = host(N.ibm_probe_loads(plan, dev(X), dev(u), dev(p), 0.4, 0.02, acc=dev(acc)))
    code, flags = N.ip_plan_status(plan)
    assert flags & N.IP_STATUS_DEGENERATE and not flags & N.IP_STATUS_NONFINITE
    fa = np.asarray(wl.faces)
    area = 0.5 * np.linalg.norm(np.cross(X[fa[:, 1]] - X[fa[:, 0]], X[fa[:, 2]] - X[fa[:, 0]]),
                                axis=1)
    dead = area == 0.0
    # the collapsed face has an exactly zero edge vector, so no normal; its
    # neighbour across the collapsed edge has two equal edge vectors, whose
    # cross product with fused multiply-adds is a rounding residue rather
    # than zero: a vanishing area and load
    assert dead.sum() == 2 and dead[11]
    assert np.array_equal(got[11], np.zeros(3))
    assert np.abs(got[dead]).max() <= 1e-12 * np.abs(got[~dead]).max()
    keep = np.flatnonzero(~dead)
    sub = types.SimpleNamespace(faces=fa[keep], closed=[1], face_off=[0, keep.size])
    want = O.probe_loads(sub, X, wl.grid, u, p, 0.4, 0.02, acc=acc[keep])
    assert rel_inf(got[keep], want) <= TOL["f64"]
    empty = W._assemble([], "empty", wl.grid, 1e-4, 1, "f64", (1.0, 1.0, 1.0, 1.0))
    plan = N.Plan(empty, empty.grid, "f64")
    z = torch.zeros(0, 3, dtype=torch.float64, device=DEV)
    out = N.ibm_probe_loads(plan, z, dev(u), dev(p), 0.4, 0.02)
    assert out.shape == (0, 3)
    assert N.ip_plan_status(plan)[0] == N.IP_OK


def test_probe_loads_ventricle_full_size_sampled():
    """The ventricle workload at full size (a closed shell and two open
    leaflets, 240 000 faces, 384 x 384 x 512): one- and two-sided probes on
    4000 sampled faces of each kind against the oracle."""
    say("probe loads ventricle full size")
    wl = W.config3()
    u, p, acc = probe_inputs(wl, "f64")
    plan = N.Plan(wl, wl.grid, "f64")
    got = host(N.ibm_probe_loads(plan, dev(wl.X), dev(u), dev(p), 0.4, 1e-3, acc=dev(acc)))
    code, flags = N.ip_plan_status(plan)
    assert code == N.IP_OK, flags
    fo = np.asarray(wl.face_off)
    rng = np.random.default_rng(6)
    for b in range(wl.n_bodies):
        pick = np.sort(rng.choice(np.arange(fo[b], fo[b + 1]), min(4000, fo[b + 1] - fo[b]),
                                  replace=False))
        sub = types.SimpleNamespace(faces=np.asarray(wl.faces)[pick], closed=[wl.closed[b]],
                                    face_off=[0, pick.size])
        want = O.probe_loads(sub, wl.X, wl.grid, u, p, 0.4, 1e-3, acc=acc[pick])
        e = rel_inf(got[pick], want)
        say(f"  body {b} ({'closed' if wl.closed[b] else 'open'}): {e:.2e}")
        assert e <= TOL["f64"]


def test_mls_ventricle_full_size():
    """MLS interpolation on sampled markers and spreading of every marker's
    force, compared point by point over the whole field, on the full-size
    ventricle, whose 100 002-node shell runs as patches."""
    say("mls ventricle full size")
    wl = W.config3()
    alpha = 0.4
    u = wl.velocity()
    plan = N.Plan(wl, wl.grid, "f64")
    assert plan.patched_bodies > 0
    X = dev(wl.X)
    U = host(N.ibm_interp_mls(plan, X, dev(u), alpha))
    Cc, Af = O.centroids(wl, wl.X)
    pick = np.random.default_rng(19).choice(wl.n_faces, 4000, replace=False)
    e_u = rel_inf(U[pick], O.interp_mls(Cc[pick], wl.grid, u, alpha))
    Fm = np.random.default_rng(20).normal(size=(wl.n_faces, 3))
    f = torch.zeros(u.shape, dtype=torch.float64, device=DEV)
    N.ibm_spread_mls(plan, X, dev(Fm), alpha, f)
    code, flags = N.ip_plan_status(plan)
    assert code == N.IP_OK, flags
    say("  gpu done; oracle spreading ...")
    f_want = O.spread_mls(Cc, Af, Fm, wl.grid, alpha)
    e_f = rel_inf(host(f), f_want)
    say(f"  U sampled {e_u:.2e}  f {e_f:.2e} (whole field)")
    assert e_u <= TOL["f64"] and e_f <= TOL["f64"]
