"""Seeded synthetic inputs for the interaction-potential + immersed-boundary path.

This module builds the *inputs* of the method and nothing else: triangulated
meshes (icospheres, a geodesic ellipsoidal shell, flat leaflet patches), their
connectivity in the layout the library takes, body placement, node noise,
elastic constants and staggered (MAC) velocity fields.  It computes none of the
method's quantities (no lengths, angles, areas, volumes, forces or transfer
weights); the test oracle and the GPU library each derive those on their own.

Connectivity follows the auxiliary arrays of the paper's data-structure section
(Section 5: vertices of a face, the four vertices of the two faces sharing an
edge): ``faces[F][3]`` lists each triangle counter-clockwise seen from outside,
``edges4[E][4]`` holds ``(v1, v2, v3, v4)`` where ``(v1, v2)`` is the edge,
``v3`` closes the face ``(v1, v2, v3)`` and ``v4`` closes the face
``(v2, v1, v4)``; a missing face (open boundary) is ``-1``.

Seeds: ``numpy.random.SeedSequence(1000 + config).spawn(4)`` gives one stream
each for placement, node noise, the velocity field and calibration targets.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------
# Meshes
# ----------------------------------------------------------------------------


def _icosahedron():
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array(
        [[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
         [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
         [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    f = np.array(
        [[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
         [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
         [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
         [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, f


def icosphere(level: int):
    """Unit icosphere by repeated 4-way midpoint subdivision, projected to the
    unit sphere.  Returns ``(verts[V,3] float64, faces[F,3] int32)`` with
    V = 10*4**L + 2, F = 20*4**L, faces counter-clockwise from outside."""
    v, f = _icosahedron()
    verts = [tuple(p) for p in v]
    for _ in range(level):
        cache: dict[tuple[int, int], int] = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                p = (np.array(verts[a]) + np.array(verts[b])) * 0.5
                p /= np.linalg.norm(p)
                idx = len(verts)
                verts.append(tuple(p))
                cache[key] = idx
            return idx

        nf = np.empty((4 * len(f), 3), dtype=np.int64)
        for n, (a, b, c) in enumerate(f):
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf[4 * n + 0] = (a, ab, ca)
            nf[4 * n + 1] = (b, bc, ab)
            nf[4 * n + 2] = (c, ca, bc)
            nf[4 * n + 3] = (ab, bc, ca)
        f = nf
    return np.asarray(verts, dtype=np.float64), f.astype(np.int32)


def geodesic_sphere(freq: int):
    """Class-I geodesic subdivision of the icosahedron with frequency ``freq``:
    every icosahedron face is split into freq**2 triangles and the points are
    projected to the unit sphere.  V = 10 f^2 + 2, E = 30 f^2, F = 20 f^2."""
    v0, f0 = _icosahedron()
    index: dict[tuple, int] = {}
    pts: list[np.ndarray] = []

    def node(corners, weights):
        key = tuple(sorted((c, w) for c, w in zip(corners, weights) if w > 0))
        idx = index.get(key)
        if idx is None:
            p = sum(w * v0[c] for c, w in key) / float(freq)
            p = p / np.linalg.norm(p)
            idx = len(pts)
            pts.append(p)
            index[key] = idx
        return idx

    faces = []
    for (a, b, c) in f0:
        grid = {}
        for i in range(freq + 1):
            for j in range(freq + 1 - i):
                grid[(i, j)] = node((a, b, c), (freq - i - j, i, j))
        for i in range(freq):
            for j in range(freq - i):
                p00, p10, p01 = grid[(i, j)], grid[(i + 1, j)], grid[(i, j + 1)]
                faces.append((p00, p10, p01))
                if i + j + 1 < freq:
                    p11 = grid[(i + 1, j + 1)]
                    faces.append((p10, p11, p01))
    return np.asarray(pts, dtype=np.float64), np.asarray(faces, dtype=np.int32)


def flat_patch(nu: int, nv: int, width: float, height: float):
    """Open rectangular membrane of ``nu x nv`` quads, each split into two
    triangles, in the local (s, t) plane: s along ``width``, t along ``height``.
    Returns ``(st[(nu+1)(nv+1), 2], faces[2 nu nv, 3])``; node (i, j) has id
    ``j*(nu+1) + i`` so row j = nv is the top edge."""
    s = np.linspace(0.0, width, nu + 1)
    t = np.linspace(0.0, height, nv + 1)
    ss, tt = np.meshgrid(s, t)
    st = np.stack([ss.ravel(), tt.ravel()], axis=1)
    faces = []
    for j in range(nv):
        for i in range(nu):
            a = j * (nu + 1) + i
            b, c, d = a + 1, a + nu + 1, a + nu + 2
            faces.append((a, b, d))
            faces.append((a, d, c))
    return st, np.asarray(faces, dtype=np.int32)


def edges4_from_faces(faces: np.ndarray) -> np.ndarray:
    """``edges4[E][4]`` for one body from its faces (local or global ids).
    Each undirected edge appears once, oriented as the half-edge ``v1 -> v2``
    with ``v1 < v2`` when both half-edges exist, else as its only half-edge."""
    faces = np.asarray(faces, dtype=np.int64)
    half = {}
    for (a, b, c) in faces:
        for (p, q, w) in ((a, b, c), (b, c, a), (c, a, b)):
            if (p, q) in half:
                raise ValueError(f"non-manifold or inconsistently oriented edge ({p},{q})")
            half[(p, q)] = w
    rows = []
    seen = set()
    for (p, q), w in half.items():
        key = (min(p, q), max(p, q))
        if key in seen:
            continue
        seen.add(key)
        back = half.get((q, p), -1)
        if back == -1:
            rows.append((p, q, w, -1))
        elif p < q:
            rows.append((p, q, w, back))
        else:
            rows.append((q, p, back, w))
    rows.sort(key=lambda r: (min(r[0], r[1]), max(r[0], r[1])))
    return np.asarray(rows, dtype=np.int32).reshape(-1, 4)


# ----------------------------------------------------------------------------
# Batches of bodies
# ----------------------------------------------------------------------------


@dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    h: float

    @property
    def extent(self):
        return (self.nx * self.h, self.ny * self.h, self.nz * self.h)


@dataclass
class Workload:
    """All inputs of one configuration.  Arrays are host numpy arrays; global
    node ids index ``X``; bodies are contiguous ranges given by the offsets."""
    name: str
    X: np.ndarray            # [N,3] float64 current positions
    Xref: np.ndarray         # [N,3] float64 reference (stress-free) positions
    faces: np.ndarray        # [F,3] int32 global ids
    edges4: np.ndarray       # [E,4] int32 global ids, -1 = no wing
    node_off: np.ndarray     # [B+1] int64
    edge_off: np.ndarray     # [B+1] int64
    face_off: np.ndarray     # [B+1] int64
    closed: np.ndarray       # [B] uint8 (1 = closed surface with volume term)
    pinned: np.ndarray       # [N] uint8
    ks: np.ndarray           # [B] float64
    kb: np.ndarray
    kA: np.ndarray
    kV: np.ndarray
    mass: np.ndarray         # [B] float64 node mass
    grid: Grid
    dt: float
    steps: int
    precision: str           # "f64" or "f32"
    field_seed: np.random.SeedSequence | None = None
    field_kind: str = "fourier"
    targets: np.ndarray | None = None   # [B] Taylor-deformation targets (calibration)
    extra: dict = field(default_factory=dict)

    @property
    def n_bodies(self):
        return len(self.node_off) - 1

    @property
    def n_nodes(self):
        return int(self.node_off[-1])

    @property
    def n_edges(self):
        return int(self.edge_off[-1])

    @property
    def n_faces(self):
        return int(self.face_off[-1])

    def velocity(self, dtype=np.float64):
        """Staggered velocity field ``u[3][nz][ny][nx]``."""
        return velocity_field(self.grid, self.field_seed, kind=self.field_kind,
                              dtype=dtype)


def _assemble(bodies, name, grid, dt, steps, precision, consts, mass=1.0):
    """bodies: list of dicts with local 'X', 'Xref', 'faces', 'closed',
    optional 'pinned' (local node mask)."""
    Xs, Xr, Fs, Es, pins = [], [], [], [], []
    node_off = [0]
    edge_off = [0]
    face_off = [0]
    closed = []
    e4cache: dict[int, np.ndarray] = {}
    for b in bodies:
        base = node_off[-1]
        key = id(b["faces"])
        e4 = e4cache.get(key)
        if e4 is None:
            e4 = e4cache[key] = edges4_from_faces(b["faces"])
        e4g = np.where(e4 >= 0, e4 + base, -1).astype(np.int32)
        Xs.append(b["X"])
        Xr.append(b["Xref"])
        Fs.append((b["faces"] + base).astype(np.int32))
        Es.append(e4g)
        pins.append(b.get("pinned", np.zeros(len(b["X"]), np.uint8)))
        node_off.append(base + len(b["X"]))
        edge_off.append(edge_off[-1] + len(e4))
        face_off.append(face_off[-1] + len(b["faces"]))
        closed.append(1 if b["closed"] else 0)
    B = len(bodies)
    ks, kb, kA, kV = consts
    if B == 0:
        Xs, Xr = [np.zeros((0, 3))], [np.zeros((0, 3))]
        Fs, Es = [np.zeros((0, 3), np.int32)], [np.zeros((0, 4), np.int32)]
        pins = [np.zeros(0, np.uint8)]
    return Workload(
        name=name,
        X=np.ascontiguousarray(np.concatenate(Xs)),
        Xref=np.ascontiguousarray(np.concatenate(Xr)),
        faces=np.ascontiguousarray(np.concatenate(Fs)),
        edges4=np.ascontiguousarray(np.concatenate(Es)),
        node_off=np.asarray(node_off, np.int64),
        edge_off=np.asarray(edge_off, np.int64),
        face_off=np.asarray(face_off, np.int64),
        closed=np.asarray(closed, np.uint8),
        pinned=np.ascontiguousarray(np.concatenate(pins).astype(np.uint8)),
        ks=np.broadcast_to(np.asarray(ks, np.float64), (B,)).copy(),
        kb=np.broadcast_to(np.asarray(kb, np.float64), (B,)).copy(),
        kA=np.broadcast_to(np.asarray(kA, np.float64), (B,)).copy(),
        kV=np.broadcast_to(np.asarray(kV, np.float64), (B,)).copy(),
        mass=np.broadcast_to(np.asarray(mass, np.float64), (B,)).copy(),
        grid=grid, dt=dt, steps=steps, precision=precision)


def _periodic_centres(rng, n, box, dmin, max_tries=2_000_000):
    """Rejection sampling of ``n`` centres in a periodic box with minimum
    periodic distance ``dmin`` (cell-list accelerated)."""
    box = np.asarray(box, np.float64)
    ncell = np.maximum((box // dmin).astype(int), 1)
    cells: dict[tuple, list] = {}
    out = []
    tries = 0
    while len(out) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("placement failed: box too crowded")
        p = rng.random(3) * box
        c = tuple((p / box * ncell).astype(int) % ncell)
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    key = ((c[0] + dx) % ncell[0], (c[1] + dy) % ncell[1],
                           (c[2] + dz) % ncell[2])
                    for q in cells.get(key, ()):
                        d = p - q
                        d -= box * np.round(d / box)
                        if d @ d < dmin * dmin:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            out.append(p)
            cells.setdefault(c, []).append(p)
    return np.asarray(out)


def _streams(config: int, k: int = 4):
    return [np.random.default_rng(s)
            for s in np.random.SeedSequence(1000 + config).spawn(k)]


def config0():
    """One level-3 icosphere drop, radius 0.1, at the centre of the unit box;
    node noise sigma = 0.01 r; 64^3 grid; dt = 1e-4; one FP64 step."""
    place, noise, _, _ = _streams(0)
    v, f = icosphere(3)
    r = 0.1
    c = np.array([0.5, 0.5, 0.5])
    Xref = c + r * v
    X = Xref + noise.normal(0.0, 0.01 * r, size=Xref.shape)
    wl = _assemble([dict(X=X, Xref=Xref, faces=f, closed=True)], "drop_L3_64",
                   Grid(64, 64, 64, 1.0 / 64), 1e-4, 1, "f64",
                   (1.0, 0.01, 0.1, 1.0))
    wl.field_seed = np.random.SeedSequence(1000).spawn(4)[2]
    return wl


def suspension(n_bodies=1000, level=4, r=0.02, n=256, sigma_rel=0.02,
               precision="f64", config=1, steps=100):
    """``n_bodies`` identical icosphere drops placed without overlap (minimum
    periodic centre distance 2.2 r) in the unit periodic box."""
    place, noise, _, targ = _streams(config)
    v, f = icosphere(level)
    centres = _periodic_centres(place, n_bodies, (1.0, 1.0, 1.0), 2.2 * r)
    bodies = []
    for c in centres:
        Xref = c + r * v
        X = Xref + noise.normal(0.0, sigma_rel * r, size=Xref.shape)
        bodies.append(dict(X=X, Xref=Xref, faces=f, closed=True))
    wl = _assemble(bodies, f"suspension_{n_bodies}xL{level}_{n}", Grid(n, n, n, 1.0 / n),
                   1e-4, steps, precision, (1.0, 0.01, 0.1, 1.0))
    wl.field_seed = np.random.SeedSequence(1000 + config).spawn(4)[2]
    wl.extra["centres"] = centres
    wl.extra["radius"] = r
    return wl


def config1(n_bodies=1000, precision="f64"):
    """1000 level-4 drops (2562 nodes each), r = 0.02, sigma = 0.02 r,
    256^3 grid, 100 steps."""
    return suspension(n_bodies=n_bodies, precision=precision, config=1)


def config2(n_bodies=4096, n=512):
    """Uneven batch: icosphere levels uniform in {2,3,4,5}, radii uniform in
    [0.008, 0.03], current shape = reference sphere stretched about its centre
    by per-axis factors uniform in [1, 1.5]; per-body constants log-uniform
    over a 10x range about (1, 0.01, 0.1, 1); uniform centres; FP32."""
    place, noise, _, _ = _streams(2)
    meshes = {L: icosphere(L) for L in (2, 3, 4, 5)}
    levels = place.integers(2, 6, size=n_bodies)
    radii = place.uniform(0.008, 0.03, size=n_bodies)
    centres = place.random((n_bodies, 3))
    stretch = noise.uniform(1.0, 1.5, size=(n_bodies, 3))
    logk = noise.uniform(-0.5, 0.5, size=(n_bodies, 4))
    bodies = []
    for b in range(n_bodies):
        v, f = meshes[int(levels[b])]
        Xref = centres[b] + radii[b] * v
        X = centres[b] + radii[b] * v * stretch[b]
        bodies.append(dict(X=X, Xref=Xref, faces=f, closed=True))
    k = np.array([1.0, 0.01, 0.1, 1.0])[None, :] * 10.0 ** logk
    wl = _assemble(bodies, f"uneven_{n_bodies}_{n}", Grid(n, n, n, 1.0 / n), 1e-4, 1,
                   "f32", (k[:, 0], k[:, 1], k[:, 2], k[:, 3]))
    wl.field_seed = np.random.SeedSequence(1002).spawn(4)[2]
    wl.extra["levels"] = levels
    return wl


def config3(freq=100, leaflet_quads=100, noise_rel=0.0, cells_per_unit=256):
    """Ventricle-like membranes: closed prolate ellipsoidal shell (semi-axes
    0.3, 0.3, 0.8; geodesic frequency 100 -> 200 000 triangles) centred in a
    1.5 x 1.5 x 2.0 box (384 x 384 x 512, h = 1/256), plus two open flat
    leaflets (100 x 100 quads, 0.24 x 0.12) in the planes x = 0.75 +- 0.08 with
    their top edge at z = 1.6; the top row of each leaflet is pinned.  The
    velocity is an axial Gaussian jet plus random-Fourier noise."""
    place, noise, _, _ = _streams(3)
    h = 1.0 / cells_per_unit
    grid = Grid(cells_per_unit * 3 // 2, cells_per_unit * 3 // 2, cells_per_unit * 2, h)
    centre = np.array([0.75, 0.75, 1.0])
    v, f = geodesic_sphere(freq)
    Xref_shell = centre + v * np.array([0.3, 0.3, 0.8])
    st, fl = flat_patch(leaflet_quads, leaflet_quads, 0.24, 0.12)
    bodies = [dict(X=Xref_shell.copy(), Xref=Xref_shell, faces=f, closed=True)]
    for side in (-1.0, 1.0):
        x = np.full(len(st), 0.75 + side * 0.08)
        y = 0.75 - 0.12 + st[:, 0]
        z = 1.6 - 0.12 + st[:, 1]
        Xr = np.stack([x, y, z], axis=1)
        fl_o = fl if side > 0 else fl[:, [0, 2, 1]]
        pin = np.zeros(len(st), np.uint8)
        pin[-(leaflet_quads + 1):] = 1          # top row t = height
        bodies.append(dict(X=Xr.copy(), Xref=Xr, faces=fl_o, closed=False, pinned=pin))
    wl = _assemble(bodies, "ventricle_shell_leaflets", grid, 1e-4, 100, "f64",
                   (1.0, 0.01, 0.1, 1.0))
    if noise_rel > 0:
        wl.X = wl.X + noise.normal(0.0, noise_rel * h, size=wl.X.shape) * (1 - wl.pinned[:, None])
    wl.field_seed = np.random.SeedSequence(1003).spawn(4)[2]
    wl.field_kind = "jet"
    return wl


def config4(n_bodies=1000):
    """Calibration: the config-1 suspension with Taylor-deformation targets
    uniform in [0.05, 0.2]; 10 steps."""
    wl = suspension(n_bodies=n_bodies, config=1, steps=10)
    targ = _streams(4)[3]
    wl.targets = targ.uniform(0.05, 0.2, size=wl.n_bodies)
    wl.name = f"calibration_{n_bodies}xL4_256"
    return wl


def small_suspension(n_bodies=4, level=2, n=32, r=0.06, seed_config=11,
                     precision="f64"):
    """A few small drops on a coarse grid: the seconds-scale parity case."""
    return suspension(n_bodies=n_bodies, level=level, r=r, n=n, sigma_rel=0.02,
                      precision=precision, config=seed_config, steps=1)


def subset(wl, ids):
    """The bodies ``ids`` of a workload as a workload of their own (node ids
    rebased); everything per body is sliced, nothing is recomputed."""
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


CONFIGS = {0: config0, 1: config1, 2: config2, 3: config3, 4: config4}

# ----------------------------------------------------------------------------
# Velocity fields on the staggered grid
# ----------------------------------------------------------------------------

#: Offsets (in cells) of the three MAC lattices: u_x lives at (i, j+1/2, k+1/2) h,
#: u_y at (i+1/2, j, k+1/2) h, u_z at (i+1/2, j+1/2, k) h.
MAC_OFFSETS = ((0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0))


def fourier_modes(seed, extent, n_modes=8, amp=0.1, kmax=4):
    rng = np.random.default_rng(seed)
    modes = []
    while len(modes) < n_modes:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if not k.any():
            continue
        kw = 2.0 * np.pi * k / np.asarray(extent)      # wave vector
        a = rng.normal(size=3)
        a -= (a @ kw) / (kw @ kw) * kw                 # divergence-free: a . k = 0
        a /= np.linalg.norm(a)
        phi = rng.uniform(0.0, 2.0 * np.pi)
        modes.append((kw, amp * a, phi))
    return modes


def velocity_field(grid: Grid, seed, kind="fourier", dtype=np.float64, zchunk=32):
    """Sample the velocity field on the three MAC lattices -> u[3][nz][ny][nx].

    fourier: sum of 8 divergence-free modes a_m sin(k_m . x + phi_m), |a_m| = 0.1.
    jet:     u_z += exp(-rho^2 / 0.1^2) about the box's vertical axis, plus the
             Fourier noise above."""
    nx, ny, nz, h = grid.nx, grid.ny, grid.nz, grid.h
    ext = grid.extent
    modes = fourier_modes(seed, ext)
    u = np.zeros((3, nz, ny, nx), dtype=dtype)
    for d in range(3):
        ox, oy, oz = MAC_OFFSETS[d]
        xs = (np.arange(nx) + ox) * h
        ys = (np.arange(ny) + oy) * h
        zs = (np.arange(nz) + oz) * h
        for z0 in range(0, nz, zchunk):
            zz = zs[z0:z0 + zchunk]
            acc = np.zeros((len(zz), ny, nx), dtype=np.float64)
            for kw, a, phi in modes:
                if a[d] == 0.0:
                    continue
                ex = np.exp(1j * (kw[0] * xs + phi))
                ey = np.exp(1j * kw[1] * ys)
                ez = np.exp(1j * kw[2] * zz)
                acc += a[d] * (ez[:, None, None] * ey[None, :, None] * ex[None, None, :]).imag
            if kind == "jet" and d == 2:
                cx, cy = ext[0] / 2, ext[1] / 2
                rho2 = (xs[None, :] - cx) ** 2 + (ys[:, None] - cy) ** 2
                acc += np.exp(-rho2 / 0.01)[None, :, :]
            u[d, z0:z0 + zchunk] = acc
    return u


def velocity_at(points, grid: Grid, seed, kind="fourier"):
    """The analytic field (same modes) at arbitrary points [N,3]."""
    modes = fourier_modes(seed, grid.extent)
    out = np.zeros_like(points, dtype=np.float64)
    for kw, a, phi in modes:
        out += np.sin(points @ kw + phi)[:, None] * a[None, :]
    if kind == "jet":
        ext = grid.extent
        rho2 = (points[:, 0] - ext[0] / 2) ** 2 + (points[:, 1] - ext[1] / 2) ** 2
        out[:, 2] += np.exp(-rho2 / 0.01)
    return out
