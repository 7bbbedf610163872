"""Shared helpers of the GPU parity tests: device transfer, oracle-side
reference marshalling and the normwise error measures."""
import numpy as np
import torch

import oracle as O
from paper_1612_03399_amd import native as N
from paper_1612_03399_amd import workload as W
from paper_1612_03399_amd.workload import subset  # noqa: F401  (re-exported for the tests)

DEV = "cuda"


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def gpu_reference_from_oracle(ref, precision):
    """The oracle's reference state in the library's layout (theta0 given by
    its cosine and sine), rounded to the plan precision."""
    dt = N.real_dtype(precision)
    cs0 = np.stack([np.cos(ref.theta0), np.sin(ref.theta0)], axis=1)
    return N.Reference(dev(ref.l0, dt), dev(cs0, dt), dev(ref.A0, dt), dev(ref.V0, torch.float64))


def oracle_reference_as_seen(ref, precision):
    """What the oracle must use to see the same (rounded) reference as the GPU."""
    if precision == "f64":
        return ref
    f = lambda a: np.asarray(a, np.float32).astype(np.float64)
    th = np.arctan2(f(np.sin(ref.theta0)), f(np.cos(ref.theta0)))
    return O.Reference(f(ref.l0), th, f(ref.A0), ref.V0.copy())


def constants(wl):
    return N.Constants.from_arrays(wl.ks, wl.kb, wl.kA, wl.kV, wl.mass, DEV)


def per_body_rel(y, yhat, node_off):
    """max over bodies of ||y - yhat||_inf / ||yhat||_inf (rows = nodes)."""
    worst = 0.0
    for b in range(len(node_off) - 1):
        s = slice(node_off[b], node_off[b + 1])
        den = np.abs(yhat[s]).max()
        if den == 0:
            num = np.abs(y[s]).max()
            worst = max(worst, num)
            continue
        worst = max(worst, np.abs(y[s] - yhat[s]).max() / den)
    return worst


def rel_inf(y, yhat):
    den = np.abs(yhat).max()
    return np.abs(y - yhat).max() / (den if den > 0 else 1.0)


def elem_rel(y, yhat):
    y, yhat = np.asarray(y), np.asarray(yhat)
    den = np.maximum(np.abs(yhat), 1e-300)
    return (np.abs(y - yhat) / den).max() if y.size else 0.0


TOL = {"f64": 1e-12, "f32": 1e-5}


def step_error(wl, Xg, Xo, X0, tol):
    """Worst body's |Xg - Xo|_inf / (tol |Xo - X0|_inf + 2 ulp(|X0|)); <= 1 passes.
    The new positions are rounded to the spacing of |X| on both sides, so the
    bar is the relative tolerance on the step plus two ulps of the positions."""
    worst = 0.0
    for b in range(len(wl.node_off) - 1):
        s = slice(int(wl.node_off[b]), int(wl.node_off[b + 1]))
        if s.start == s.stop:
            continue
        dx = np.abs(Xo[s] - X0[s]).max()
        ulp = np.spacing(np.abs(X0[s]).max())
        worst = max(worst, np.abs(Xg[s] - Xo[s]).max() / (tol * dx + 2 * ulp))
    return worst


def body_spheres(wl):
    c = np.empty((wl.n_bodies, 3))
    r = np.empty(wl.n_bodies)
    for b in range(wl.n_bodies):
        x = wl.X[wl.node_off[b]:wl.node_off[b + 1]]
        c[b] = x.mean(axis=0)
        r[b] = np.sqrt(((x - c[b]) ** 2).sum(axis=1).max())
    return c, r


def support_mask(X, grid):
    """Points of the three lattices within the 27-point supports of X."""
    n = np.array([grid.nx, grid.ny, grid.nz])
    m = np.zeros((3, grid.nz, grid.ny, grid.nx), bool)
    for d in range(3):
        off = np.array(W.MAC_OFFSETS[d])
        c = np.floor(X / grid.h - off + 0.5).astype(np.int64)
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    i = (c + np.array([dx, dy, dz])) % n
                    m[d, i[:, 2], i[:, 1], i[:, 0]] = True
    return m


def near_bodies(wl, sample, extra_cells=3.0):
    """Sorted ids of the bodies whose grid support can reach that of a body in
    `sample` (bounding spheres about the node mean, grown by extra_cells grid
    spacings; unit periodic box)."""
    c, r = body_spheres(wl)
    reach = r + extra_cells * wl.grid.h
    near = set()
    for b in sample:
        d = c - c[b]
        d -= np.round(d)
        near |= set(np.flatnonzero(np.sqrt((d * d).sum(axis=1)) < reach + reach[b]).tolist())
    return sorted(near)


def energy_error(Wg, Wo, Vg, Vo, wl, V0, tol):
    """Worst ratio (<= 1 passes) of the energy differences [B][4] to their bar.
    W_s, W_b and W_a: elementwise tol.  W_v = kV (V - V0)^2 / (2 V0) depends on
    the body's volume alone and is conditioned by V / |V - V0|: a volume
    difference dV between two FP64 summation orders moves it by
    |dW_v/dV| dV = kV |V - V0| / V0 dV, so its bar is tol W_v plus that
    propagation of the measured volume difference (V itself is checked at
    tol on its own)."""
    Wg, Wo = np.asarray(Wg, np.float64), np.asarray(Wo, np.float64)
    bar = tol * np.abs(Wo)
    closed = np.asarray(wl.closed) == 1
    dV = np.abs(np.asarray(Vg) - np.asarray(Vo))
    V0 = np.where(closed, np.asarray(V0, np.float64), 1.0)
    slope = np.asarray(wl.kV) * np.abs(np.asarray(Vo) - V0) / V0
    bar[:, 3] += np.where(closed, slope * dV * (1 + tol), 0.0)
    diff = np.abs(Wg - Wo)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(bar > 0, diff / np.where(bar > 0, bar, 1.0), np.where(diff > 0, np.inf, 0.0))
    return float(r.max()) if r.size else 0.0

