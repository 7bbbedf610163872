"""FP64 CPU oracle for the interaction-potential + immersed-boundary step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_1612_03399_amd``) and never imports it.

The arithmetic lives in plain C (``oracle.c`` / ``oracle_core.inc``), serial
loops in element order; this module compiles it with gcc, marshals numpy arrays
through ctypes, and writes out the reverse-mode recursion over time steps from
the C primitives.  Citations (paper sections / equations) are in the C source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "oracle_core.inc"),
        os.path.join(_HERE, "oracle_mls.inc")]
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (always, when ``force``)."""
    newest = max(os.path.getmtime(s) for s in _SRC)
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < newest:
        tmp = _SO + f".tmp{os.getpid()}"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fcx-limited-range",
             "-Wall", "-Wno-unused-function", "-Wno-maybe-uninitialized", "-o", tmp, _SRC[0], "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_SO)
        d, i64, i32, u8 = (C.POINTER(C.c_double), C.POINTER(C.c_int64),
                           C.POINTER(C.c_int32), C.POINTER(C.c_uint8))
        L.orc_phi.restype = C.c_double
        L.orc_phi.argtypes = [C.c_double]
        L.orc_geometry.argtypes = [C.c_int, i64, i64, i32, d, d, d]
        L.orc_reference.argtypes = [C.c_int, i64, i64, i64, i32, i32, d, d, d, d, d]
        L.orc_forces.argtypes = [C.c_int, i64, i64, i64, i32, i32, u8, d, d, d, d, d, d,
                                 d, d, d, d, d, d]
        L.orc_forces_jvp.argtypes = [C.c_int, i64, i64, i64, i32, i32, u8, d, d, d, d, d, d,
                                     d, d, d]
        L.orc_interp.argtypes = [C.c_int64, d, C.c_int, C.c_int, C.c_int, C.c_double, d, d]
        L.orc_interp_jac.argtypes = [C.c_int64, d, C.c_int, C.c_int, C.c_int, C.c_double, d, d]
        L.orc_spread.argtypes = [C.c_int64, d, d, C.c_int, C.c_int, C.c_int, C.c_double, d]
        L.orc_step.argtypes = [C.c_int, i64, i64, i64, i32, i32, u8, u8, d, d, d, d, d, d, d,
                               d, C.c_int, C.c_int, C.c_int, C.c_double, d, d, C.c_double,
                               d, d, d, d]
        L.orc_taylor.argtypes = [C.c_int, i64, d, d, d]
        L.orc_taylor_loss_grad.restype = C.c_double
        L.orc_taylor_loss_grad.argtypes = [C.c_int, i64, d, d, d]
        L.orc_centroids.argtypes = [C.c_int64, i32, d, d, d]
        L.orc_mls_shape.restype = C.c_int
        L.orc_mls_shape.argtypes = [C.c_int64, d, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                    C.c_double, i64, d]
        L.orc_interp_mls.restype = C.c_int
        L.orc_interp_mls.argtypes = [C.c_int64, d, C.c_int, C.c_int, C.c_int, C.c_double,
                                     C.c_double, d, d]
        L.orc_spread_mls.restype = C.c_int
        L.orc_spread_mls.argtypes = [C.c_int64, d, d, d, C.c_int, C.c_int, C.c_int, C.c_double,
                                     C.c_double, d]
        L.orc_centroid_to_nodes.argtypes = [C.c_int64, C.c_int64, i32, d, d]
        L.orc_probe_loads.restype = C.c_int
        L.orc_probe_loads.argtypes = [C.c_int, i64, u8, i32, d, C.c_int, C.c_int, C.c_int,
                                      C.c_double, C.c_double, d, d, d, C.c_double, d]
        L.orc_direct_forcing_mls.restype = C.c_int
        L.orc_direct_forcing_mls.argtypes = [C.c_int64, d, d, d, C.c_int, C.c_int, C.c_int,
                                             C.c_double, C.c_double, d, C.c_double, d, d]
        _lib = L
    return _lib


def _p(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _mesh_args(m):
    no = np.ascontiguousarray(m.node_off, np.int64)
    eo = np.ascontiguousarray(m.edge_off, np.int64)
    fo = np.ascontiguousarray(m.face_off, np.int64)
    fa = np.ascontiguousarray(m.faces, np.int32)
    e4 = np.ascontiguousarray(m.edges4, np.int32)
    return no, eo, fo, fa, e4


def _k(m, k=None):
    if k is None:
        k = np.stack([m.ks, m.kb, m.kA, m.kV])
    return _f64(np.asarray(k).reshape(4, -1))


class Reference:
    """Reference state: l0[E], theta0[E], A0[F], V0[B] (float64)."""

    def __init__(self, l0, theta0, A0, V0):
        self.l0, self.theta0, self.A0, self.V0 = l0, theta0, A0, V0


def phi(r: float) -> float:
    return lib().orc_phi(float(r))


def geometry(m, X):
    no, eo, fo, fa, e4 = _mesh_args(m)
    B = len(no) - 1
    X = _f64(X)
    V = np.zeros(B)
    A = np.zeros(B)
    lib().orc_geometry(B, _p(no, C.c_int64), _p(fo, C.c_int64), _p(fa, C.c_int32),
                       _p(X, C.c_double), _p(V, C.c_double), _p(A, C.c_double))
    return V, A


def reference(m, Xref=None) -> Reference:
    no, eo, fo, fa, e4 = _mesh_args(m)
    B = len(no) - 1
    Xr = _f64(m.Xref if Xref is None else Xref)
    l0 = np.zeros(int(eo[-1]))
    th = np.zeros(int(eo[-1]))
    A0 = np.zeros(int(fo[-1]))
    V0 = np.zeros(B)
    lib().orc_reference(B, _p(no, C.c_int64), _p(eo, C.c_int64), _p(fo, C.c_int64),
                        _p(fa, C.c_int32), _p(e4, C.c_int32), _p(Xr, C.c_double),
                        _p(l0, C.c_double), _p(th, C.c_double), _p(A0, C.c_double),
                        _p(V0, C.c_double))
    return Reference(l0, th, A0, V0)


def _ew(m, ew):
    """Per-edge weights [E][2] on (ks, kb) as float64, or None (all 1)."""
    if ew is None:
        return None
    ew = _f64(np.asarray(ew).reshape(-1, 2))
    assert ew.shape[0] == int(np.asarray(m.edge_off)[-1])
    return ew


def forces(m, X, ref: Reference, k=None, families=False, ew=None):
    """Returns dict(F, V, A, W[B,4], Ffam[4,N,3] if families).  ew[E][2]:
    per-edge weights on (ks, kb), None for all 1."""
    no, eo, fo, fa, e4 = _mesh_args(m)
    B = len(no) - 1
    N = int(no[-1])
    X = _f64(X)
    kk = _k(m, k)
    F = np.zeros((N, 3))
    Ff = np.zeros((4, N, 3)) if families else None
    V = np.zeros(B)
    A = np.zeros(B)
    W = np.zeros((B, 4))
    cl = np.ascontiguousarray(m.closed, np.uint8)
    lib().orc_forces(B, _p(no, C.c_int64), _p(eo, C.c_int64), _p(fo, C.c_int64),
                     _p(fa, C.c_int32), _p(e4, C.c_int32), _p(cl, C.c_uint8),
                     _p(X, C.c_double), _p(_f64(ref.l0), C.c_double),
                     _p(_f64(ref.theta0), C.c_double), _p(_f64(ref.A0), C.c_double),
                     _p(_f64(ref.V0), C.c_double), _p(kk, C.c_double),
                     _p(_ew(m, ew), C.c_double), _p(F, C.c_double),
                     _p(Ff, C.c_double), _p(V, C.c_double), _p(A, C.c_double),
                     _p(W, C.c_double))
    out = dict(F=F, V=V, A=A, W=W)
    if families:
        out["Ffam"] = Ff
    return out


def forces_jvp(m, X, dX, ref: Reference, k=None, ew=None):
    """(dF/dX) dX by the complex step; equal to the VJP (dF/dX symmetric)."""
    no, eo, fo, fa, e4 = _mesh_args(m)
    B = len(no) - 1
    X = _f64(X)
    dX = _f64(dX)
    dF = np.zeros_like(X)
    cl = np.ascontiguousarray(m.closed, np.uint8)
    lib().orc_forces_jvp(B, _p(no, C.c_int64), _p(eo, C.c_int64), _p(fo, C.c_int64),
                         _p(fa, C.c_int32), _p(e4, C.c_int32), _p(cl, C.c_uint8),
                         _p(X, C.c_double), _p(dX, C.c_double), _p(_f64(ref.l0), C.c_double),
                         _p(_f64(ref.theta0), C.c_double), _p(_f64(ref.A0), C.c_double),
                         _p(_f64(ref.V0), C.c_double), _p(_k(m, k), C.c_double),
                         _p(_ew(m, ew), C.c_double), _p(dF, C.c_double))
    return dF


def _grid(grid):
    return int(grid.nx), int(grid.ny), int(grid.nz), float(grid.h)


def interp(X, grid, u):
    X = _f64(X)
    u = _f64(u)
    U = np.zeros_like(X)
    nx, ny, nz, h = _grid(grid)
    lib().orc_interp(len(X), _p(X, C.c_double), nx, ny, nz, h, _p(u, C.c_double),
                     _p(U, C.c_double))
    return U


def interp_jac(X, grid, u):
    """J[l, d, e] = dU_d(X_l)/dX_{l,e}."""
    X = _f64(X)
    u = _f64(u)
    J = np.zeros((len(X), 3, 3))
    nx, ny, nz, h = _grid(grid)
    lib().orc_interp_jac(len(X), _p(X, C.c_double), nx, ny, nz, h, _p(u, C.c_double),
                         _p(J, C.c_double))
    return J


def spread(X, Fn, grid, f=None):
    X = _f64(X)
    Fn = _f64(Fn)
    nx, ny, nz, h = _grid(grid)
    if f is None:
        f = np.zeros((3, nz, ny, nx))
    assert f.dtype == np.float64 and f.flags.c_contiguous
    lib().orc_spread(len(X), _p(X, C.c_double), _p(Fn, C.c_double), nx, ny, nz, h,
                     _p(f, C.c_double))
    return f


def step(m, X, ref: Reference, u, dt, f=None, k=None, ew=None):
    """One explicit step; returns dict(X=new X, F, U, V, A, f)."""
    no, eo, fo, fa, e4 = _mesh_args(m)
    B = len(no) - 1
    Xn = _f64(X).copy()
    u = _f64(u)
    F = np.zeros_like(Xn)
    U = np.zeros_like(Xn)
    V = np.zeros(B)
    A = np.zeros(B)
    nx, ny, nz, h = _grid(m.grid)
    cl = np.ascontiguousarray(m.closed, np.uint8)
    pn = np.ascontiguousarray(m.pinned, np.uint8)
    ms = _f64(m.mass)
    lib().orc_step(B, _p(no, C.c_int64), _p(eo, C.c_int64), _p(fo, C.c_int64),
                   _p(fa, C.c_int32), _p(e4, C.c_int32), _p(cl, C.c_uint8),
                   _p(pn, C.c_uint8), _p(ms, C.c_double), _p(Xn, C.c_double),
                   _p(_f64(ref.l0), C.c_double), _p(_f64(ref.theta0), C.c_double),
                   _p(_f64(ref.A0), C.c_double), _p(_f64(ref.V0), C.c_double),
                   _p(_k(m, k), C.c_double), _p(_ew(m, ew), C.c_double), nx, ny, nz, h,
                   _p(u, C.c_double),
                   _p(f, C.c_double), float(dt), _p(F, C.c_double), _p(U, C.c_double),
                   _p(V, C.c_double), _p(A, C.c_double))
    return dict(X=Xn, F=F, U=U, V=V, A=A, f=f)


def taylor(m, X):
    no = np.ascontiguousarray(m.node_off, np.int64)
    B = len(no) - 1
    X = _f64(X)
    D = np.zeros(B)
    ev = np.zeros((B, 3))
    lib().orc_taylor(B, _p(no, C.c_int64), _p(X, C.c_double), _p(D, C.c_double),
                     _p(ev, C.c_double))
    return D, ev


def taylor_loss_grad(m, X, Dstar):
    no = np.ascontiguousarray(m.node_off, np.int64)
    B = len(no) - 1
    X = _f64(X)
    g = np.zeros_like(X)
    Ds = _f64(Dstar)
    loss = lib().orc_taylor_loss_grad(B, _p(no, C.c_int64), _p(X, C.c_double),
                                      _p(Ds, C.c_double), _p(g, C.c_double))
    return loss, g


def node_body(m):
    no = np.asarray(m.node_off)
    return np.repeat(np.arange(len(no) - 1), np.diff(no))


def rollout_grad(m, X0, ref: Reference, u, dt, steps, Dstar, k=None, ew=None):
    """Loss after ``steps`` explicit steps and its gradient by reverse mode.

    Forward: X^{n+1} = X^n + M (dt U(X^n) + dt^2/m F(X^n; k)), M = not pinned.
    Reverse, with P = M lambda^{n+1}:
      lambda^n = lambda^{n+1} + dt J_U(X^n)^T P + (dt^2/m) (dF/dX)(X^n) P
      g_k[s, b] += (dt^2/m_b) sum_{l in b} F_s(X^n; k_s = 1) . P_l
      g_u += dt h^3 spread(P)      (interpolation's adjoint is spreading)
    Returns dict(loss, gX0[N,3], gk[4,B], gu, X_final)."""
    kk = _k(m, k)
    nb = node_body(m)
    mask = (1 - np.asarray(m.pinned, np.float64))[:, None]
    c2 = (dt * dt / np.asarray(m.mass, np.float64))[nb][:, None]
    Xs = [_f64(X0).copy()]
    for _ in range(steps):
        Xs.append(step(m, Xs[-1], ref, u, dt, None, kk, ew)["X"])
    loss, lam = taylor_loss_grad(m, Xs[-1], Dstar)
    B = len(m.node_off) - 1
    gk = np.zeros((4, B))
    h = m.grid.h
    gu = np.zeros((3, m.grid.nz, m.grid.ny, m.grid.nx))
    for n in range(steps - 1, -1, -1):
        Xn = Xs[n]
        P = mask * lam
        J = interp_jac(Xn, m.grid, u)
        # each family's force is linear in its own constant: dF_s/dk_s is the
        # family's force at unit constants (defined also where k_s = 0)
        fu = forces(m, Xn, ref, np.ones_like(kk), families=True, ew=ew)
        dF = forces_jvp(m, Xn, P, ref, kk, ew)
        lam = lam + dt * np.einsum("lde,ld->le", J, P) + c2 * dF
        for s in range(4):
            contrib = (fu["Ffam"][s] * P).sum(axis=1) * c2[:, 0]
            gk[s] += np.bincount(nb, contrib, minlength=B)
        spread(Xn, P, m.grid, gu_tmp := np.zeros_like(gu))
        gu += dt * h ** 3 * gu_tmp
    return dict(loss=loss, gX0=lam, gk=gk, gu=gu, X_final=Xs[-1])


# ---- MLS transfer at the triangle centroids (Section 2.2; oracle_mls.inc) ----

def centroids(m, X):
    """Face centroids C[F][3] (the Lagrangian markers) and face areas A[F]."""
    fa = np.ascontiguousarray(m.faces, np.int32)
    X = _f64(X)
    Cc = np.zeros((len(fa), 3))
    Af = np.zeros(len(fa))
    lib().orc_centroids(len(fa), _p(fa, C.c_int32), _p(X, C.c_double), _p(Cc, C.c_double),
                        _p(Af, C.c_double))
    return Cc, Af


def mls_shape(P, grid, d, alpha):
    """Support indices idx[M][27] (flat in one lattice) and MLS shape
    functions phi[M][27] of positions P on lattice d."""
    P = _f64(P)
    M = len(P)
    idx = np.zeros((M, 27), np.int64)
    phi = np.zeros((M, 27))
    nx, ny, nz, h = _grid(grid)
    bad = lib().orc_mls_shape(M, _p(P, C.c_double), int(d), nx, ny, nz, h, float(alpha),
                              _p(idx, C.c_int64), _p(phi, C.c_double))
    assert bad == 0, f"{bad} singular moment matrices"
    return idx, phi


def interp_mls(P, grid, u, alpha):
    """U[M][3] at positions P, component d from lattice d of u."""
    P = _f64(P)
    u = _f64(u)
    U = np.zeros((len(P), 3))
    nx, ny, nz, h = _grid(grid)
    bad = lib().orc_interp_mls(len(P), _p(P, C.c_double), nx, ny, nz, h, float(alpha),
                               _p(u, C.c_double), _p(U, C.c_double))
    assert bad == 0, f"{bad} singular moment matrices"
    return U


def spread_mls(P, Am, Fm, grid, alpha, f=None):
    """f += MLS spreading of the marker force densities Fm[M][3] (marker
    areas Am[M]) with the force-conserving factor c_l."""
    P = _f64(P)
    nx, ny, nz, h = _grid(grid)
    if f is None:
        f = np.zeros((3, nz, ny, nx))
    assert f.dtype == np.float64 and f.flags.c_contiguous
    bad = lib().orc_spread_mls(len(P), _p(P, C.c_double), _p(_f64(Am), C.c_double),
                               _p(_f64(Fm), C.c_double), nx, ny, nz, h, float(alpha),
                               _p(f, C.c_double))
    assert bad == 0, f"{bad} singular moment matrices"
    return f


def centroid_to_nodes(m, Fc):
    """Vertex forces: each vertex takes one third of the centroid force of
    every face it belongs to."""
    fa = np.ascontiguousarray(m.faces, np.int32)
    N = int(np.asarray(m.node_off)[-1])
    Fn = np.zeros((N, 3))
    lib().orc_centroid_to_nodes(N, len(fa), _p(fa, C.c_int32), _p(_f64(Fc), C.c_double),
                                _p(Fn, C.c_double))
    return Fn


def direct_forcing_mls(P, Am, Vb, grid, u, alpha, dt, f=None):
    """Direct forcing at the markers: Fm = (Vb - MLS interp of u) / dt, and
    f += MLS spreading of Fm.  Returns (Fm, f)."""
    P = _f64(P)
    nx, ny, nz, h = _grid(grid)
    if f is None:
        f = np.zeros((3, nz, ny, nx))
    Fm = np.zeros((len(P), 3))
    bad = lib().orc_direct_forcing_mls(len(P), _p(P, C.c_double), _p(_f64(Am), C.c_double),
                                       _p(_f64(Vb), C.c_double), nx, ny, nz, h, float(alpha),
                                       _p(_f64(u), C.c_double), float(dt), _p(Fm, C.c_double),
                                       _p(f, C.c_double))
    assert bad == 0, f"{bad} singular moment matrices"
    return Fm, f


def probe_loads(m, X, grid, u, p, alpha, mu, acc=None):
    """External loads Fext[F][3] on every face from normal probes of length h:
    pressure (cell-centred field p[nz][ny][nx]) and viscous stress mu (G + G^T)
    from the MLS fits at the probe ends; one probe on closed bodies, two on
    open ones; acc[F][3] the marker acceleration (None: zero)."""
    fo = np.ascontiguousarray(m.face_off, np.int64)
    fa = np.ascontiguousarray(m.faces, np.int32)
    cl = np.ascontiguousarray(m.closed, np.uint8)
    nx, ny, nz, h = _grid(grid)
    Fext = np.zeros((len(fa), 3))
    bad = lib().orc_probe_loads(len(fo) - 1, _p(fo, C.c_int64), _p(cl, C.c_uint8),
                                _p(fa, C.c_int32), _p(_f64(X), C.c_double), nx, ny, nz, h,
                                float(alpha), _p(_f64(u), C.c_double), _p(_f64(p), C.c_double),
                                None if acc is None else _p(_f64(acc), C.c_double), float(mu),
                                _p(Fext, C.c_double))
    assert bad == 0, f"{bad} singular moment matrices"
    return Fext
