"""GPU parity: the HIP library (through its C-ABI) against the FP64 oracle,
element by element on the same seeded inputs.  FP64 plans must agree to 1e-12
relative (per-body normwise for node arrays, global normwise for grid fields,
elementwise for per-body scalars), FP32 plans to 1e-5 against the oracle run
on the same FP32-rounded inputs."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1612_03399_amd import native as N
from paper_1612_03399_amd import workload as W

from gpu_common import (DEV, TOL, constants, dev, elem_rel, energy_error,
                        gpu_reference_from_oracle, host, oracle_reference_as_seen, per_body_rel,
                        rel_inf)

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def sparse_icosahedra():
    """Level-0 icosahedra much larger than a cell: their bounding-box tile does
    not fit the step kernel's LDS and the fused path falls back to direct
    grid access."""
    return W.suspension(n_bodies=3, level=0, r=0.2, n=48, sigma_rel=0.02, config=12, steps=1)


CASES = {
    "drop_L3_64": lambda: W.config0(),
    "sparse_L0_48": sparse_icosahedra,
    "four_L2_32": lambda: W.small_suspension(4, 2, 32),
    # bench-shaped bodies (level 4, radius 5.12 h): more spreading work items
    # than a workgroup's lanes, every fused-kernel loop takes several turns
    "four_L4_128": lambda: W.small_suspension(4, 4, 128, r=0.04),
    "uneven_small": lambda: W.config2(n_bodies=24, n=64),
    # level-4 drops of radius 1.9 h: ~55 nodes per occupied cell, so a
    # cell's nodes are spread by several work items
    "crowded_L4_32": lambda: W.small_suspension(2, 4, 32, r=0.06),
    "ventricle_small": lambda: W.config3(freq=12, leaflet_quads=10, noise_rel=0.2,
                                         cells_per_unit=64),
    # a 16 002-node shell: the fused step splits it into patches with halos
    "ventricle_patched": lambda: W.config3(freq=40, leaflet_quads=30, noise_rel=0.2,
                                           cells_per_unit=96),
    # 300 units: two full rounds of the chunked deal of units to the XCDs
    # (128 units each) and a ragged tail of 44 in plain order
    "many_L1_64": lambda: W.small_suspension(300, 1, 64, r=0.03),
}


def build(case, precision):
    wl = CASES[case]()
    ref = O.reference(wl)
    return wl, ref


def run_forces(wl, ref, precision):
    plan = N.Plan(wl, wl.grid, precision)
    gref = gpu_reference_from_oracle(ref, precision)
    k = constants(wl)
    X = dev(wl.X)
    V = torch.empty(wl.n_bodies, dtype=torch.float64, device=DEV)
    A = torch.empty_like(V)
    Wt = torch.empty(wl.n_bodies, 4, dtype=torch.float64, device=DEV)
    F = N.ip_forces(plan, X, gref, k, V=V, A=A, W=Wt)
    code, flags = N.ip_plan_status(plan)
    return plan, host(F).astype(np.float64), host(V), host(A), host(Wt), code


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", list(CASES))
def test_forces_parity(case, precision):
    say("forces", case, precision)
    wl, ref = build(case, precision)
    oref = oracle_reference_as_seen(ref, precision)
    want = O.forces(wl, wl.X, oref)
    plan, F, V, A, Wg, code = run_forces(wl, ref, precision)
    assert code == N.IP_OK
    tol = TOL[precision]
    assert per_body_rel(F, want["F"], wl.node_off) <= tol
    # V is FP64 in both precisions
    assert elem_rel(V[wl.closed == 1], want["V"][wl.closed == 1]) <= 1e-12
    assert elem_rel(A, want["A"]) <= tol
    assert energy_error(Wg, want["W"], V, want["V"], wl, oref.V0,
                        1e-12 if precision == "f64" else 1e-6) <= 1.0


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_reference_from(precision):
    say("reference_from", precision)
    wl = W.config3(freq=12, leaflet_quads=10, cells_per_unit=64)
    ref = O.reference(wl)
    plan = N.Plan(wl, wl.grid, precision)
    g = N.ip_reference_from(plan, dev(wl.Xref))
    torch.cuda.synchronize()
    tol = 1e-14 if precision == "f64" else 1e-7
    assert elem_rel(host(g.l0), ref.l0) <= tol
    assert elem_rel(host(g.A0), ref.A0) <= tol
    assert elem_rel(host(g.V0)[wl.closed == 1], ref.V0[wl.closed == 1]) <= 1e-14
    cs = host(g.cs0).astype(np.float64)
    assert np.abs(cs[:, 0] - np.cos(ref.theta0)).max() <= tol * 4
    assert np.abs(cs[:, 1] - np.sin(ref.theta0)).max() <= tol * 4


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", ["drop_L3_64", "four_L2_32", "ventricle_small"])
def test_interp_spread_parity(case, precision):
    say("interp/spread", case, precision)
    wl, ref = build(case, precision)
    dt = N.real_dtype(precision)
    u = wl.velocity()
    if precision == "f32":
        u = u.astype(np.float32).astype(np.float64)
    plan = N.Plan(wl, wl.grid, precision)
    X = dev(wl.X)
    ud = dev(u, dt)
    U = host(N.ibm_interp(plan, X, ud)).astype(np.float64)
    want_U = O.interp(wl.X, wl.grid, u)
    assert per_body_rel(U, want_U, wl.node_off) <= TOL[precision]
    rng = np.random.default_rng(3)
    Fn = rng.normal(size=wl.X.shape)
    if precision == "f32":
        Fn = Fn.astype(np.float32).astype(np.float64)
    f = torch.zeros(3, wl.grid.nz, wl.grid.ny, wl.grid.nx, dtype=dt, device=DEV)
    N.ibm_spread(plan, X, dev(Fn, dt), f)
    want_f = O.spread(wl.X, Fn, wl.grid)
    assert rel_inf(host(f).astype(np.float64), want_f) <= TOL[precision]


def check_step(case, precision, bound, options=None):
    wl, ref = build(case, precision)
    dt_ = N.real_dtype(precision)
    u = wl.velocity()
    if precision == "f32":
        u = u.astype(np.float32).astype(np.float64)
    oref = oracle_reference_as_seen(ref, precision)
    f_want = np.zeros_like(u)
    want = O.step(wl, wl.X, oref, u, wl.dt, f_want)
    plan = N.Plan(wl, wl.grid, precision, options)
    X = dev(wl.X)
    f = torch.zeros(u.shape, dtype=dt_, device=DEV)
    V = torch.empty(wl.n_bodies, dtype=torch.float64, device=DEV)
    gref = gpu_reference_from_oracle(ref, precision)
    if bound:
        N.ip_plan_bind_reference(plan, gref)
        gref = None
    N.ip_step(plan, X, gref, constants(wl), dev(u, dt_), f, wl.dt, V=V)
    code, _ = N.ip_plan_status(plan)
    assert code == N.IP_OK
    # X_new = X + dX is rounded to the spacing of |X| on both sides, so the
    # bar is the relative tolerance on dX plus two ulps of the positions
    Xg, Xo = host(X), want["X"]
    for b in range(wl.n_bodies):
        s = slice(wl.node_off[b], wl.node_off[b + 1])
        dx = np.abs(Xo[s] - wl.X[s]).max()
        ulp = np.spacing(np.abs(wl.X[s]).max())
        assert np.abs(Xg[s] - Xo[s]).max() <= TOL[precision] * dx + 2 * ulp
    assert rel_inf(host(f).astype(np.float64), f_want) <= TOL[precision]
    Vg = host(V)
    assert elem_rel(Vg[wl.closed == 1], want["V"][wl.closed == 1]) <= 1e-12
    pin = wl.pinned == 1
    if pin.any():
        assert np.array_equal(host(X)[pin], wl.X[pin])
    return plan


@pytest.mark.parametrize("bound", [False, True], ids=["explicit_ref", "bound_ref"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", list(CASES))
def test_step_parity(case, precision, bound):
    """One step; with a bound reference the fused step reads the packed,
    conflict-ordered element records instead of the caller's arrays."""
    say("step", case, precision, "bound" if bound else "explicit")
    check_step(case, precision, bound)


#: launch shapes the autotuner chooses between (all compute the same step)
LAUNCH_SHAPES = {
    "t384": {"threads": 384},
    "t384_small_units": {"threads": 384, "unit_nodes": 640, "patch_owned": 384,
                         "tile_bytes": 12288},
    "t768_tile8k": {"tile_bytes": 8192},
    "patch256": {"unit_nodes": 768, "patch_owned": 256},
    "patch512": {"unit_nodes": 1536, "patch_owned": 512},
    "t384_two_per_cu": {"threads": 384, "wg_per_cu": 2},
    "t256_three_per_cu": {"threads": 256, "wg_per_cu": 3},
    "t256_small_units": {"threads": 256, "wg_per_cu": 2, "unit_nodes": 384, "patch_owned": 128},
    "t128_four_per_cu": {"threads": 128, "wg_per_cu": 4, "patch_owned": 256},
    "t128_six_per_cu": {"threads": 128, "wg_per_cu": 6, "patch_owned": 128},
}


@pytest.mark.parametrize("shape", list(LAUNCH_SHAPES))
@pytest.mark.parametrize("case", ["four_L4_128", "uneven_small", "ventricle_patched",
                                  "many_L1_64"])
def test_step_parity_launch_shapes(case, shape):
    say("step shape", case, shape)
    opts = LAUNCH_SHAPES[shape]
    plan = check_step(case, "f64", True, opts)
    # without a thread count the plan puts units of at most 1536 nodes on
    # 384-thread workgroups and larger ones on 768
    assert plan.fused and plan.step_threads == opts.get("threads", plan.step_threads)
    assert plan.step_threads in (128, 256, 384, 768)


def test_autotune_choice_computes_the_step(tmp_path, monkeypatch):
    """The autotuner's staged search (reference computed from the reference
    positions with its first plan) times distinct launch shapes of all three
    stages, caches its choice (the second call is a lookup returning the same
    options), and the shape it picks computes the step to parity."""
    from paper_1612_03399_amd import autotune as AT
    monkeypatch.setenv("IPIBM_TUNE_CACHE", str(tmp_path / "tune.json"))
    say("autotune four_L4_128")
    wl = CASES["four_L4_128"]()
    u = dev(wl.velocity())
    args = (wl, wl.grid, "f64", dev(wl.X), None, constants(wl), u, wl.dt)
    opts, results, info = AT.autotune(*args, steps=2, warmup=1, Xref=dev(wl.Xref))
    assert info["cache"] == "miss"
    assert len(results) >= 3 and all(r["ms"] > 0 for r in results)
    assert {r["stage"] for r in results} >= {1, 2}
    assert opts in [r["options"] for r in results]
    again, results2, info2 = AT.autotune(*args, steps=2, warmup=1, Xref=dev(wl.Xref))
    assert info2["cache"] == "hit" and again == opts and results2 == results
    check_step("four_L4_128", "f64", True, opts)


def test_forces_deterministic():
    say("determinism")
    wl, ref = build("four_L2_32", "f64")
    _, F1, *_ = run_forces(wl, ref, "f64")
    _, F2, *_ = run_forces(wl, ref, "f64")
    assert np.array_equal(F1, F2)


def test_spread_adjoint_of_interp_on_gpu():
    say("adjointness")
    wl = W.small_suspension(4, 2, 32)
    plan = N.Plan(wl, wl.grid, "f64")
    rng = np.random.default_rng(0)
    u = rng.normal(size=(3, 32, 32, 32))
    Fn = rng.normal(size=wl.X.shape)
    X = dev(wl.X)
    U = host(N.ibm_interp(plan, X, dev(u)))
    f = torch.zeros(u.shape, dtype=torch.float64, device=DEV)
    N.ibm_spread(plan, X, dev(Fn), f)
    lhs = (host(f) * u).sum() * wl.grid.h ** 3
    rhs = (Fn * U).sum()
    assert abs(lhs - rhs) <= 1e-12 * np.abs(Fn * U).sum()


def test_empty_batch_and_zero_force_reference():
    say("edge cases")
    wl = W.config0()
    empty = W._assemble([], "empty", wl.grid, 1e-4, 1, "f64", (1.0, 1.0, 1.0, 1.0))
    plan = N.Plan(empty, empty.grid, "f64")
    z = torch.zeros(0, 3, dtype=torch.float64, device=DEV)
    e = torch.zeros(0, dtype=torch.float64, device=DEV)
    ref = N.Reference(e, torch.zeros(0, 2, dtype=torch.float64, device=DEV), e, e)
    k = N.Constants(e, e, e, e, e)
    F = N.ip_forces(plan, z, ref, k)
    assert F.shape == (0, 3)
    # at the reference configuration the forces vanish (GPU-computed reference)
    plan = N.Plan(wl, wl.grid, "f64")
    Xr = dev(wl.Xref)
    g = N.ip_reference_from(plan, Xr)
    F = host(N.ip_forces(plan, Xr, g, constants(wl)))
    F_cur = host(N.ip_forces(plan, dev(wl.X), g, constants(wl)))
    assert np.abs(F).max() <= 1e-13 * np.abs(F_cur).max()


def test_degenerate_face_sets_status():
    say("degenerate")
    wl = W.config0()
    ref = O.reference(wl)
    X = wl.X.copy()
    a, b, c = wl.faces[7]
    X[c] = X[a]          # collapse one triangle (and the edges touching it)
    plan = N.Plan(wl, wl.grid, "f64")
    N.ip_forces(plan, dev(X), gpu_reference_from_oracle(ref, "f64"), constants(wl))
    code, flags = N.ip_plan_status(plan)
    assert code in (N.IP_ERR_DEGENERATE, N.IP_ERR_NONFINITE)
    assert flags & N.IP_STATUS_DEGENERATE
    code, flags = N.ip_plan_status(plan)      # cleared by the read
    assert code == N.IP_OK and flags == 0


def test_bound_reference_entry_points():
    """Forces, derivatives and the reverse step accept the bound reference;
    without one bound, a NULL reference is an argument error."""
    say("bound reference")
    wl, ref = build("four_L2_32", "f64")
    plan = N.Plan(wl, wl.grid, "f64")
    gref = gpu_reference_from_oracle(ref, "f64")
    k = constants(wl)
    X = dev(wl.X)
    with pytest.raises(N.IpibmError) as e:
        N.ip_forces(plan, X, None, k)
    assert e.value.code == N.IP_ERR_ARG
    F1 = host(N.ip_forces(plan, X, gref, k))
    N.ip_plan_bind_reference(plan, gref)
    F2 = host(N.ip_forces(plan, X, None, k))
    assert np.array_equal(F1, F2)
    dX = dev(np.random.default_rng(4).normal(size=wl.X.shape))
    assert np.array_equal(host(N.ip_forces_jvp(plan, X, dX, gref, k)),
                          host(N.ip_forces_jvp(plan, X, dX, None, k)))
    # rebinding replaces the reference: bind the current shape, forces vanish
    g2 = N.ip_reference_from(plan, X)
    N.ip_plan_bind_reference(plan, g2)
    F3 = host(N.ip_forces(plan, X, None, k))
    assert np.abs(F3).max() <= 1e-13 * np.abs(F1).max()


def test_large_body_is_patched():
    say("patches")
    wl = CASES["ventricle_patched"]()
    plan = N.Plan(wl, wl.grid, "f64")
    assert plan.fused and plan.patched_bodies == 1
    assert plan.n_units > wl.n_bodies
