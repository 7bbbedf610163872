"""ctypes binding of ``libipibm.so`` (declared in ``include/ipibm.h``).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Device arrays are torch tensors (torch supplies device memory and
streams); host mesh arrays are numpy arrays.  If the library is not built this
module raises at import -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch  # loads the HIP runtime the library binds to

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("IPIBM_LIB", os.path.join(PKG, "libipibm.so"))

IP_OK, IP_ERR_ARG, IP_ERR_HIP, IP_ERR_DEGENERATE, IP_ERR_NONFINITE, IP_ERR_OOM, \
    IP_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
IP_F64, IP_F32 = 0, 1
IP_STATUS_DEGENERATE, IP_STATUS_NONFINITE = 0x1, 0x2
_NAMES = {0: "IP_OK", -1: "IP_ERR_ARG", -2: "IP_ERR_HIP", -3: "IP_ERR_DEGENERATE",
          -4: "IP_ERR_NONFINITE", -5: "IP_ERR_OOM", -6: "IP_ERR_UNSUPPORTED"}


class IpibmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class ip_mesh(C.Structure):
    _fields_ = [("n_bodies", C.c_int32), ("node_off", C.c_void_p), ("edge_off", C.c_void_p),
                ("face_off", C.c_void_p), ("faces", C.c_void_p), ("edges4", C.c_void_p),
                ("closed", C.c_void_p), ("pinned", C.c_void_p)]


class ip_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("h", C.c_double)]


class ip_plan_options(C.Structure):
    _fields_ = [("unit_nodes", C.c_int32), ("patch_owned", C.c_int32), ("tile_bytes", C.c_int32),
                ("threads", C.c_int32), ("wg_per_cu", C.c_int32)]


class ip_reference(C.Structure):
    _fields_ = [("l0", C.c_void_p), ("cs0", C.c_void_p), ("A0", C.c_void_p),
                ("V0", C.c_void_p)]


class ip_constants(C.Structure):
    _fields_ = [("ks", C.c_void_p), ("kb", C.c_void_p), ("kA", C.c_void_p),
                ("kV", C.c_void_p), ("mass", C.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built (python paper_1612_03399_amd/build.py)")
    lib = C.CDLL(LIB_PATH)
    vp, i32, d = C.c_void_p, C.c_int32, C.c_double
    sig = {
        "ip_plan_create": [C.POINTER(vp), C.POINTER(ip_mesh), C.POINTER(ip_grid), i32],
        "ip_plan_create_ex": [C.POINTER(vp), C.POINTER(ip_mesh), C.POINTER(ip_grid), i32,
                              C.POINTER(ip_plan_options)],
        "ip_plan_destroy": [vp],
        "ip_plan_sizes": [vp, C.POINTER(C.c_int64)],
        "ip_plan_properties": [vp, C.POINTER(C.c_int64)],
        "ip_reference_from": [vp, vp, vp, vp, vp, vp, vp],
        "ip_forces": [vp, vp, C.POINTER(ip_reference), C.POINTER(ip_constants), vp, vp, vp, vp,
                      vp],
        "ip_forces_noalloc": [vp, vp, C.POINTER(ip_reference), C.POINTER(ip_constants), vp, vp,
                              vp, vp, vp],
        "ibm_interp": [vp, vp, vp, vp, vp],
        "ibm_spread": [vp, vp, vp, vp, vp],
        "ip_step": [vp, vp, C.POINTER(ip_reference), C.POINTER(ip_constants), vp, vp, d, vp,
                    vp, vp],
        "ip_plan_status": [vp, vp, C.POINTER(C.c_uint32)],
        "ip_forces_jvp": [vp, vp, vp, C.POINTER(ip_reference), C.POINTER(ip_constants), vp, vp],
        "ip_plan_bind_reference": [vp, C.POINTER(ip_reference), vp],
        "ip_plan_bind_edge_weights": [vp, vp, vp],
        "ibm_interp_vjp": [vp, vp, vp, vp, vp, vp, vp],
        "ip_step_vjp": [vp, vp, C.POINTER(ip_reference), C.POINTER(ip_constants), vp, d, vp, vp,
                        vp, vp, vp],
        "ip_taylor": [vp, vp, vp, vp, vp, vp, vp],
        "ibm_interp_mls": [vp, vp, vp, d, vp, vp],
        "ibm_spread_mls": [vp, vp, vp, d, vp, vp],
        "ip_centroid_to_nodes": [vp, vp, vp, vp],
        "ibm_direct_forcing_mls": [vp, vp, vp, vp, d, d, vp, vp, vp],
        "ibm_probe_loads": [vp, vp, vp, vp, vp, d, d, vp, vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.ip_last_error.restype = C.c_char_p
    lib.ip_last_error.argtypes = []
    return lib


LIB = _load()


def _check(code):
    if code != IP_OK:
        raise IpibmError(code, LIB.ip_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if not t.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return t.data_ptr()
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    raise TypeError(type(t))


def _refp(ref):
    """Pointer to an ip_reference, or NULL for the reference bound to the plan."""
    return None if ref is None else C.byref(ref.struct())


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def real_dtype(precision: str):
    return torch.float64 if precision == "f64" else torch.float32


@dataclass
class Reference:
    """Reference state on the device: l0[E], cs0[E,2], A0[F] (real), V0[B] (double)."""
    l0: torch.Tensor
    cs0: torch.Tensor
    A0: torch.Tensor
    V0: torch.Tensor

    def struct(self):
        return ip_reference(_ptr(self.l0), _ptr(self.cs0), _ptr(self.A0), _ptr(self.V0))


@dataclass
class Constants:
    """Per-body constants on the device, double[B] each."""
    ks: torch.Tensor
    kb: torch.Tensor
    kA: torch.Tensor
    kV: torch.Tensor
    mass: torch.Tensor

    def struct(self):
        return ip_constants(_ptr(self.ks), _ptr(self.kb), _ptr(self.kA), _ptr(self.kV),
                            _ptr(self.mass))

    @staticmethod
    def from_arrays(ks, kb, kA, kV, mass, device="cuda"):
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float64), device=device)
        return Constants(f(ks), f(kb), f(kA), f(kV), f(mass))


class Plan:
    """Owns an ``ip_plan``.  ``mesh`` is any object with host arrays node_off,
    edge_off, face_off, faces, edges4, closed, pinned (see ip_mesh)."""

    def __init__(self, mesh, grid=None, precision: str = "f64", options=None):
        self.precision = precision
        self.dtype = real_dtype(precision)
        self._keep = [np.ascontiguousarray(mesh.node_off, np.int64),
                      np.ascontiguousarray(mesh.edge_off, np.int64),
                      np.ascontiguousarray(mesh.face_off, np.int64),
                      np.ascontiguousarray(mesh.faces, np.int32),
                      np.ascontiguousarray(mesh.edges4, np.int32),
                      np.ascontiguousarray(mesh.closed, np.uint8),
                      None if getattr(mesh, "pinned", None) is None
                      else np.ascontiguousarray(mesh.pinned, np.uint8)]
        no, eo, fo, fa, e4, cl, pn = self._keep
        m = ip_mesh(len(no) - 1, _ptr(no), _ptr(eo), _ptr(fo), _ptr(fa), _ptr(e4), _ptr(cl),
                    _ptr(pn))
        g = None
        if grid is not None:
            g = ip_grid(int(grid.nx), int(grid.ny), int(grid.nz), float(grid.h))
            self.grid = (int(grid.nx), int(grid.ny), int(grid.nz), float(grid.h))
        else:
            self.grid = None
        h = C.c_void_p()
        self.options = dict(options or {})
        opt = ip_plan_options(int(self.options.get("unit_nodes", 0)),
                              int(self.options.get("patch_owned", 0)),
                              int(self.options.get("tile_bytes", 0)),
                              int(self.options.get("threads", 0)),
                              int(self.options.get("wg_per_cu", 0)))
        _check(LIB.ip_plan_create_ex(C.byref(h), C.byref(m), C.byref(g) if g else None,
                                     IP_F64 if precision == "f64" else IP_F32, C.byref(opt)))
        self.handle = h
        counts = (C.c_int64 * 4)()
        _check(LIB.ip_plan_sizes(h, counts))
        self.B, self.N, self.E, self.F = (int(c) for c in counts)
        props = (C.c_int64 * 6)()
        _check(LIB.ip_plan_properties(h, props))
        self.fused = bool(props[0])
        (self.largest_unit, self.tile_bytes, self.step_threads, self.n_units,
         self.patched_bodies) = (int(v) for v in props[1:])

    def close(self):
        if getattr(self, "handle", None):
            LIB.ip_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ip_plan_create(mesh, grid=None, precision="f64", options=None) -> Plan:
    """options: dict with any of unit_nodes, patch_owned, tile_bytes, threads,
    wg_per_cu (see ip_plan_options)."""
    return Plan(mesh, grid, precision, options)


def ip_reference_from(plan: Plan, Xref: torch.Tensor, stream=None) -> Reference:
    dev = Xref.device
    ref = Reference(torch.empty(plan.E, dtype=plan.dtype, device=dev),
                    torch.empty(plan.E, 2, dtype=plan.dtype, device=dev),
                    torch.empty(plan.F, dtype=plan.dtype, device=dev),
                    torch.empty(plan.B, dtype=torch.float64, device=dev))
    _check(LIB.ip_reference_from(plan.handle, _ptr(Xref), _ptr(ref.l0), _ptr(ref.cs0),
                                 _ptr(ref.A0), _ptr(ref.V0), _stream(stream)))
    return ref


def ip_forces(plan: Plan, X, ref: Reference, k: Constants, F=None, V=None, A=None, W=None,
              stream=None):
    if F is None:
        F = torch.empty(plan.N, 3, dtype=plan.dtype, device=X.device)
    r, kk = _refp(ref), k.struct()
    _check(LIB.ip_forces(plan.handle, _ptr(X), r, C.byref(kk), _ptr(F), _ptr(V),
                         _ptr(A), _ptr(W), _stream(stream)))
    return F


def ip_forces_noalloc(plan: Plan, X, ref: Reference, k: Constants, F, V=None, A=None, W=None,
                      stream=None):
    """ip_forces with its workspace in the library's static scratch: F (and
    V, A, W when wanted) must be given, so nothing is allocated here either."""
    r, kk = _refp(ref), k.struct()
    _check(LIB.ip_forces_noalloc(plan.handle, _ptr(X), r, C.byref(kk), _ptr(F), _ptr(V),
                                 _ptr(A), _ptr(W), _stream(stream)))
    return F


def ibm_interp(plan: Plan, X, u, U=None, stream=None):
    if U is None:
        U = torch.empty(plan.N, 3, dtype=plan.dtype, device=X.device)
    _check(LIB.ibm_interp(plan.handle, _ptr(X), _ptr(u), _ptr(U), _stream(stream)))
    return U


def ibm_spread(plan: Plan, X, F, f, stream=None):
    _check(LIB.ibm_spread(plan.handle, _ptr(X), _ptr(F), _ptr(f), _stream(stream)))
    return f


def ibm_interp_mls(plan: Plan, X, u, alpha, U=None, stream=None):
    """MLS interpolation to the face centroids: U[F][3] (real)."""
    if U is None:
        U = torch.empty(plan.F, 3, dtype=plan.dtype, device=X.device)
    _check(LIB.ibm_interp_mls(plan.handle, _ptr(X), _ptr(u), float(alpha), _ptr(U),
                              _stream(stream)))
    return U


def ibm_spread_mls(plan: Plan, X, Fm, alpha, f, stream=None):
    """f += MLS spreading of the centroid force densities Fm[F][3]."""
    _check(LIB.ibm_spread_mls(plan.handle, _ptr(X), _ptr(Fm), float(alpha), _ptr(f),
                              _stream(stream)))
    return f


def ibm_direct_forcing_mls(plan: Plan, X, Vb, u, alpha, dt, f, Fm=None, stream=None):
    """Direct forcing at the face centroids: Fm = (Vb - U)/dt with U the MLS
    interpolation of u, spread into f (accumulated).  Returns (Fm, f); pass
    Fm=False to skip storing the marker forces."""
    if Fm is None:
        Fm = torch.empty(plan.F, 3, dtype=plan.dtype, device=X.device)
    fm = None if Fm is False else Fm
    _check(LIB.ibm_direct_forcing_mls(plan.handle, _ptr(X), _ptr(Vb), _ptr(u), float(alpha),
                                      float(dt), _ptr(fm), _ptr(f), _stream(stream)))
    return fm, f


def ibm_probe_loads(plan: Plan, X, u, p, alpha, mu, acc=None, Fext=None, stream=None):
    """External loads Fext[F][3] on every face from normal probes (pressure
    p[nz][ny][nx] at cell centres, velocity u, marker acceleration acc[F][3])."""
    if Fext is None:
        Fext = torch.empty(plan.F, 3, dtype=plan.dtype, device=X.device)
    _check(LIB.ibm_probe_loads(plan.handle, _ptr(X), _ptr(u), _ptr(p), _ptr(acc), float(alpha),
                               float(mu), _ptr(Fext), _stream(stream)))
    return Fext


def ip_centroid_to_nodes(plan: Plan, Fc, Fn=None, stream=None):
    """Vertex forces Fn[N][3]: one third of every incident face's centroid force."""
    if Fn is None:
        Fn = torch.empty(plan.N, 3, dtype=plan.dtype, device=Fc.device)
    _check(LIB.ip_centroid_to_nodes(plan.handle, _ptr(Fc), _ptr(Fn), _stream(stream)))
    return Fn


def ip_step(plan: Plan, X, ref: Reference, k: Constants, u, f, dt, V=None, A=None,
            stream=None):
    r, kk = _refp(ref), k.struct()
    _check(LIB.ip_step(plan.handle, _ptr(X), r, C.byref(kk), _ptr(u), _ptr(f),
                       float(dt), _ptr(V), _ptr(A), _stream(stream)))
    return X


def ip_plan_status(plan: Plan, stream=None):
    flags = C.c_uint32()
    code = LIB.ip_plan_status(plan.handle, _stream(stream), C.byref(flags))
    if code not in (IP_OK, IP_ERR_DEGENERATE, IP_ERR_NONFINITE):
        _check(code)
    return code, int(flags.value)


def ip_forces_jvp(plan: Plan, X, dX, ref: Reference, k: Constants, dF=None, stream=None):
    if dF is None:
        dF = torch.empty_like(X)
    r, kk = _refp(ref), k.struct()
    _check(LIB.ip_forces_jvp(plan.handle, _ptr(X), _ptr(dX), r, C.byref(kk), _ptr(dF),
                             _stream(stream)))
    return dF


def ip_step_vjp(plan: Plan, X, ref: Reference, k: Constants, u, dt, lam_next, lam=None,
                gk=None, gu=None, stream=None):
    if lam is None:
        lam = torch.empty_like(lam_next)
    r, kk = _refp(ref), k.struct()
    _check(LIB.ip_step_vjp(plan.handle, _ptr(X), r, C.byref(kk), _ptr(u), float(dt),
                           _ptr(lam_next), _ptr(lam), _ptr(gk), _ptr(gu), _stream(stream)))
    return lam


def ip_taylor(plan: Plan, X, Dstar=None, stream=None):
    """Returns D[B], or (D, loss[B], gX[N,3]) when Dstar is given."""
    D = torch.empty(plan.B, dtype=torch.float64, device=X.device)
    if Dstar is None:
        _check(LIB.ip_taylor(plan.handle, _ptr(X), None, _ptr(D), None, None, _stream(stream)))
        return D
    loss = torch.empty_like(D)
    gX = torch.empty_like(X)
    _check(LIB.ip_taylor(plan.handle, _ptr(X), _ptr(Dstar), _ptr(D), _ptr(loss), _ptr(gX),
                         _stream(stream)))
    return D, loss, gX


def ibm_interp_vjp(plan: Plan, X, u, dU, gX=None, gu=None, want_gX=True, stream=None):
    """Adjoint of ibm_interp: returns (gX = J_U^T dU [N][3], gu); gu is
    accumulated into when given (the caller zeroes it), skipped when None."""
    if gX is None and want_gX:
        gX = torch.empty(plan.N, 3, dtype=torch.float64, device=X.device)
    _check(LIB.ibm_interp_vjp(plan.handle, _ptr(X), _ptr(u), _ptr(dU), _ptr(gX), _ptr(gu),
                              _stream(stream)))
    return gX, gu


def ip_plan_bind_edge_weights(plan: Plan, ew, stream=None):
    """Bind per-edge weights ew[E][2] (float64 device tensor: w_s, w_b on the
    body's ks, kb) for every later call on the plan; None unbinds."""
    if ew is not None:
        assert ew.dtype == torch.float64 and tuple(ew.shape) == (plan.E, 2) and ew.is_contiguous()
    _check(LIB.ip_plan_bind_edge_weights(plan.handle, _ptr(ew), _stream(stream)))


def ip_plan_bind_reference(plan: Plan, ref: Reference, stream=None):
    """Copy (and, for fused plans, pack) a reference into the plan; entry points
    then accept ref=None for it."""
    _check(LIB.ip_plan_bind_reference(plan.handle, C.byref(ref.struct()), _stream(stream)))
    plan.bound_reference = ref      # the copy is asynchronous: keep the source alive
