"""Shared helpers of the GPU parity tests: device transfer, oracle-side
reference marshalling and the normwise error measures."""
import numpy as np
import torch

import oracle as O
from paper_1612_03399_amd import native as N

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


def subset(wl, ids):
    """The bodies ``ids`` of a workload as a workload of their own (node ids
    rebased); everything per body is sliced, nothing is recomputed."""
    import dataclasses
    ids = [int(b) for b in ids]
    X, Xr, fa, e4, pn = [], [], [], [], []
    no, eo, fo = [0], [0], [0]
    for b in ids:
        n0, n1 = int(wl.node_off[b]), int(wl.node_off[b + 1])
        e0, e1 = int(wl.edge_off[b]), int(wl.edge_off[b + 1])
        f0, f1 = int(wl.face_off[b]), int(wl.face_off[b + 1])
        base = no[-1]
        X.append(wl.X[n0:n1])
        Xr.append(wl.Xref[n0:n1])
        pn.append(wl.pinned[n0:n1])
        fa.append(wl.faces[f0:f1] - n0 + base)
        e = wl.edges4[e0:e1]
        e4.append(np.where(e >= 0, e - n0 + base, -1))
        no.append(base + n1 - n0)
        eo.append(eo[-1] + e1 - e0)
        fo.append(fo[-1] + f1 - f0)
    cat = lambda a, t: np.ascontiguousarray(np.concatenate(a).astype(t))
    return dataclasses.replace(
        wl, X=cat(X, np.float64), Xref=cat(Xr, np.float64), faces=cat(fa, np.int32),
        edges4=cat(e4, np.int32), pinned=cat(pn, np.uint8),
        node_off=np.asarray(no, np.int64), edge_off=np.asarray(eo, np.int64),
        face_off=np.asarray(fo, np.int64), closed=wl.closed[ids].copy(),
        ks=wl.ks[ids].copy(), kb=wl.kb[ids].copy(), kA=wl.kA[ids].copy(),
        kV=wl.kV[ids].copy(), mass=wl.mass[ids].copy())


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
