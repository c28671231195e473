"""Seeded synthetic scenes for the CCFR hot path.

Both the oracle tests and the GPU path draw their inputs from here, so this
module only lays out meshes, masses, initial states and parameter records.
It holds none of the collision method's arithmetic: no boxes, closest points,
half-spaces, projections or constraint updates.

Every scene is a single concatenated mesh:

* ``x``         float32 [N, 3]  positions (m)
* ``v``         float32 [N, 3]  velocities (m/s)
* ``inv_mass``  float32 [N]     inverse masses (0 = static or pinned)
* ``tris``      int32   [T, 3]  triangles
* ``edges``     int32   [E, 2]  unique edges, ``a < b``, sorted lexicographically
* ``rest_x``    float32 [N, 3]  positions the stretch rest lengths are taken from

Vertices that belong to no edge and no triangle are free particles.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

CLOTH_AREAL_DENSITY = 0.1      # kg / m^2
STRAND_VERTEX_MASS = 1e-4      # kg
PARTICLE_MASS = 1e-4           # kg


@dataclass(frozen=True)
class Params:
    """Collision parameters of one mesh (metres)."""
    r: float                    # search radius and per-iteration displacement bound
    xi: float                   # offset (minimum separation)
    delta: float = 0.0          # repulsion range (response is not on this path)
    guard: float = 1e-6         # extra box padding that keeps the box test conservative
    eps_retract: float = 1e-6   # retraction margin of the projection
    eps_plesnik: float = 1e-6   # tolerance of the ERO-line update
    max_passes: int = 4         # passes of the per-vertex projection
    response: bool = False      # soft response and friction before the projection
    resp_compliance: float = 0.0  # compliance 1/k of the response constraint
    vis_width: float = 0.0      # transition width of the visibility weights (0: none)
    mu_s: float = 0.0           # static friction coefficient
    mu_k: float = 0.0           # kinetic friction coefficient


@dataclass(frozen=True)
class StepParams:
    dt: float
    gravity: tuple = (0.0, 0.0, -9.8)
    iters: int = 10
    steps: int = 10
    alpha: float = 1e-6         # stretch compliance
    early_exit: bool = False    # end a step's iterations at the convergence check
    conv_tol: float = 0.0       # shortfall (m) below which the check counts a vertex as converged


@dataclass
class Scene:
    name: str
    x: np.ndarray
    v: np.ndarray
    inv_mass: np.ndarray
    tris: np.ndarray
    edges: np.ndarray
    rest_x: np.ndarray
    params: Params
    step: StepParams
    meta: dict = field(default_factory=dict)

    @property
    def n_verts(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])

    @property
    def n_edges(self) -> int:
        return int(self.edges.shape[0])

    @property
    def n_dynamic(self) -> int:
        return int(np.count_nonzero(self.inv_mass > 0))

    def bbox_diag(self, x: np.ndarray | None = None) -> float:
        p = self.x if x is None else x
        return float(np.linalg.norm(p.max(0).astype(np.float64) - p.min(0).astype(np.float64)))

    def with_state(self, x=None, v=None, name=None) -> "Scene":
        return replace(self,
                       x=self.x if x is None else np.ascontiguousarray(x, np.float32),
                       v=self.v if v is None else np.ascontiguousarray(v, np.float32),
                       name=self.name if name is None else name)


# --------------------------------------------------------------------------
# mesh pieces
# --------------------------------------------------------------------------

class _Mesh:
    def __init__(self, x, tris, inv_mass, v=None):
        self.x = np.asarray(x, np.float64).reshape(-1, 3)
        self.tris = np.asarray(tris, np.int64).reshape(-1, 3)
        self.inv_mass = np.asarray(inv_mass, np.float64).reshape(-1)
        self.v = np.zeros_like(self.x) if v is None else np.asarray(v, np.float64)
        self.extra_edges = np.zeros((0, 2), np.int64)


def cloth_grid(n: int, side: float, center, areal_density=CLOTH_AREAL_DENSITY) -> _Mesh:
    """n x n vertices spanning side x side in the xy-plane.  Vertex (i, j) has
    index j*n + i; every quad is split on the same diagonal (i,j)-(i+1,j+1)."""
    t = np.linspace(-0.5 * side, 0.5 * side, n)
    xx, yy = np.meshgrid(t, t, indexing="xy")          # row j, column i
    x = np.stack([xx.ravel(), yy.ravel(), np.zeros(n * n)], 1) + np.asarray(center, np.float64)
    i, j = np.meshgrid(np.arange(n - 1), np.arange(n - 1), indexing="xy")
    a = (j * n + i).ravel()
    b = a + 1
    c = a + n + 1
    d = a + n
    tris = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)], 0)
    # interleave so the two triangles of one quad are adjacent in the list
    tris = tris.reshape(2, -1, 3).transpose(1, 0, 2).reshape(-1, 3)
    m = areal_density * side * side / (n * n)
    return _Mesh(x, tris, np.full(n * n, 1.0 / m))


def icosphere(level: int, radius: float, center=(0.0, 0.0, 0.0)) -> _Mesh:
    """Static icosphere: a subdivided icosahedron projected to the sphere."""
    p = (1.0 + 5 ** 0.5) / 2.0
    verts = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0),
             (0, -1, p), (0, 1, p), (0, -1, -p), (0, 1, -p),
             (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    vs = [np.asarray(v, np.float64) / np.linalg.norm(v) for v in verts]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = vs[a] + vs[b]
                vs.append(m / np.linalg.norm(m))
                cache[key] = len(vs) - 1
            return cache[key]
        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    x = np.asarray(vs) * radius + np.asarray(center, np.float64)
    return _Mesh(x, np.asarray(faces), np.zeros(len(vs)))


def ground_quad(side: float, z: float = 0.0) -> _Mesh:
    h = 0.5 * side
    x = [(-h, -h, z), (h, -h, z), (h, h, z), (-h, h, z)]
    return _Mesh(x, [(0, 1, 2), (0, 2, 3)], np.zeros(4))


def box_inward(lo, hi) -> _Mesh:
    """Closed static cuboid of 8 corners and 12 triangles facing inward."""
    (x0, y0, z0), (x1, y1, z1) = lo, hi
    x = [(x0, y0, z0), (x1, y0, z0), (x1, y1, z0), (x0, y1, z0),
         (x0, y0, z1), (x1, y0, z1), (x1, y1, z1), (x0, y1, z1)]
    quads = [(0, 1, 2, 3), (4, 7, 6, 5), (0, 4, 5, 1), (1, 5, 6, 2), (2, 6, 7, 3), (3, 7, 4, 0)]
    tris = []
    for a, b, c, d in quads:
        tris += [(a, b, c), (a, c, d)]
    return _Mesh(x, tris, np.zeros(8))


def strands_mesh(points: np.ndarray, inv_mass: np.ndarray) -> _Mesh:
    """Polylines: points [S, K, 3] -> S*K vertices and S*(K-1) segment edges."""
    s, k, _ = points.shape
    m = _Mesh(points.reshape(-1, 3), np.zeros((0, 3)), inv_mass.reshape(-1))
    base = (np.arange(s) * k)[:, None] + np.arange(k - 1)[None, :]
    m.extra_edges = np.stack([base.ravel(), base.ravel() + 1], 1)
    return m


def particles_mesh(x: np.ndarray, inv_mass: float) -> _Mesh:
    return _Mesh(x, np.zeros((0, 3)), np.full(len(x), inv_mass))


def edges_from_tris(tris: np.ndarray, extra=None) -> np.ndarray:
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]], 0) if len(tris) \
        else np.zeros((0, 2), np.int64)
    if extra is not None and len(extra):
        e = np.concatenate([e, extra], 0)
    e = np.sort(e, 1).astype(np.int64)
    if not len(e):
        return e
    # unique rows in lexicographic order, through one 64-bit key per edge
    n = int(e.max()) + 1
    k = np.unique(e[:, 0] * n + e[:, 1])
    return np.stack([k // n, k % n], 1)


def assemble(name, meshes, params, step, rest_x=None, meta=None) -> Scene:
    xs, vs, ws, ts, es = [], [], [], [], []
    off = 0
    for m in meshes:
        xs.append(m.x)
        vs.append(m.v)
        ws.append(m.inv_mass)
        ts.append(m.tris + off)
        es.append(m.extra_edges + off)
        off += len(m.x)
    x = np.concatenate(xs, 0)
    tris = np.concatenate(ts, 0).astype(np.int64)
    edges = edges_from_tris(tris, np.concatenate(es, 0))
    xf = np.ascontiguousarray(x, np.float32)
    return Scene(name=name, x=xf,
                 v=np.ascontiguousarray(np.concatenate(vs, 0), np.float32),
                 inv_mass=np.ascontiguousarray(np.concatenate(ws, 0), np.float32),
                 tris=np.ascontiguousarray(tris, np.int32),
                 edges=np.ascontiguousarray(edges, np.int32),
                 rest_x=xf.copy() if rest_x is None else np.ascontiguousarray(rest_x, np.float32),
                 params=params, step=step, meta=dict(meta or {}))


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------

def drape(n=32, side=1.0, sphere_level=3, sphere_radius=0.3, height=0.1, jitter=1e-3,
          seed=1000, r=2e-3, xi=2e-3, offset_xy=(0.0, 0.0), rot=0.0, iters=10, steps=10,
          dt=1.0 / 60.0, name=None) -> Scene:
    """Square cloth held `height` above the top of a static icosphere centred at the
    origin.  Cloth vertices get i.i.d. N(0, jitter) on every component; rest lengths
    are those of the jittered cloth."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cloth = cloth_grid(n, side, (0.0, 0.0, sphere_radius + height))
    if rot:
        c, s = math.cos(rot), math.sin(rot)
        R = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])
        cloth.x = cloth.x @ R.T
    cloth.x[:, 0] += offset_xy[0]
    cloth.x[:, 1] += offset_xy[1]
    cloth.x += rng.normal(0.0, jitter, cloth.x.shape) if np.ndim(jitter) == 0 else \
        rng.normal(0.0, 1.0, cloth.x.shape) * np.asarray(jitter)
    sph = icosphere(sphere_level, sphere_radius)
    return assemble(name or f"drape{n}", [cloth, sph], Params(r=r, xi=xi),
                    StepParams(dt=dt, iters=iters, steps=steps),
                    meta=dict(cloth_n=n, n_cloth=n * n))


# Speed knobs (cell scale, lanes per query, iterations per candidate build,
# adaptive skin) that the autotuner chose for each workload on four steps from
# the middle of its run; the benchmark times these, and the full-size GPU
# tests run the workloads with them.
BENCH_KNOBS = {
    "c0": dict(cell_scale=0.7, pair_split=9, pair_reuse=4, pair_skin=0),
    "c1": dict(cell_scale=0.7, pair_split=1, pair_reuse=3, pair_skin=0),
    "c2": dict(cell_scale=0.85, pair_split=1, pair_reuse=4, pair_skin=0),
    "c3": dict(cell_scale=0.85, pair_split=1, pair_reuse=1, pair_skin=0, direct_regions=1),
    "c5": dict(cell_scale=0.7, pair_split=9, pair_reuse=1, pair_skin=1),
    # the served stream: the serving loop's tuner (16 requests resident) on
    # the 512-request stream
    "c4": dict(cell_scale=0.7, pair_split=1, pair_reuse=2, pair_skin=0, direct_regions=1),
}


def c0() -> Scene:
    """32x32 cloth (1 m) 0.1 m above a static 642-vertex icosphere of radius 0.3 m."""
    return drape(name="c0")


def c1(n=256, side=2.0, height=0.1, vel_sigma=0.5, seed=1001) -> Scene:
    """256x256 cloth (2 m) 0.1 m above a static 4 m ground quad at z = 0, with
    i.i.d. N(0, 0.5 m/s) initial velocities per vertex and component."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cloth = cloth_grid(n, side, (0.0, 0.0, height))
    cloth.v = rng.normal(0.0, vel_sigma, cloth.x.shape)
    ground = ground_quad(2.0 * side, 0.0)
    return assemble("c1" if n == 256 else f"c1_{n}", [cloth, ground], Params(r=1e-3, xi=1e-3),
                    StepParams(dt=1.0 / 120.0, iters=20, steps=60),
                    meta=dict(cloth_n=n, n_cloth=n * n))


def folded_cloth_state(scene: Scene, seed: int, compress=0.3, amp=0.004, wavelength=0.05,
                       lift=None) -> Scene:
    """A crumpled-looking but valid state of a cloth-over-ground scene: the cloth
    (first meta['n_cloth'] vertices, a grid) is compressed along x and given a wavy
    height field, so that neighbouring rows come within the contact band while no
    part of it overlaps another in the xy-plane.  Its lowest points sit `lift` above
    z = 0 (default 1.5 xi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = scene.meta["cloth_n"]
    nc = n * n
    x = scene.x.astype(np.float64).copy()
    cx = x[:nc, 0].mean()
    x[:nc, 0] = cx + (x[:nc, 0] - cx) * compress
    ph = rng.uniform(0, 2 * np.pi, 3)
    k = 2 * np.pi / wavelength
    u, w = x[:nc, 0], x[:nc, 1]
    z = amp * (np.sin(k * u + ph[0]) + 0.5 * np.sin(0.7 * k * w + ph[1])
               + 0.25 * np.sin(0.5 * k * (u + w) + ph[2]))
    z += rng.normal(0.0, 0.05 * amp, nc)
    lift = 1.5 * scene.params.xi if lift is None else lift
    x[:nc, 2] = z - z.min() + lift
    return scene.with_state(x=x.astype(np.float32), name=scene.name + f"_folded{seed}")


def two_layers(n=12, side=0.1, gap=3e-3, jitter=4e-4, seed=7, r=1e-3, xi=1e-3,
               shift=(0.0, 0.0)) -> Scene:
    """Two dynamic cloth patches stacked `gap` apart (inside the contact band), with
    the upper one shifted in xy, plus jitter: dense vertex-face and edge-edge pairs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = cloth_grid(n, side, (0.0, 0.0, 0.0))
    b = cloth_grid(n, side, (shift[0] + 0.37 * side / (n - 1), shift[1] + 0.21 * side / (n - 1), gap))
    for m in (a, b):
        m.x += rng.normal(0.0, jitter, m.x.shape)
    return assemble(f"two_layers{n}_s{seed}", [a, b], Params(r=r, xi=xi),
                    StepParams(dt=1.0 / 120.0, iters=4, steps=2), meta=dict(cloth_n=n))


def particles_in_box(nx=6, ny=6, nz=8, spacing=9.9e-3, jitter=1.5e-3, seed=1003,
                     r=5e-3, xi=5e-3, box_margin=0.01, box_top=None) -> Scene:
    """Free particles on a jittered lattice inside a closed static inward box."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1)
    p = g.reshape(-1, 3).astype(np.float64) * spacing + box_margin
    p += rng.uniform(-jitter, jitter, p.shape)
    hi = (np.array([nx - 1, ny - 1, nz - 1]) * spacing + 2 * box_margin)
    if box_top is not None:
        hi[2] = box_top
    parts = particles_mesh(p, 1.0 / PARTICLE_MASS)
    box = box_inward((0.0, 0.0, 0.0), tuple(hi))
    return assemble(f"particles{nx}x{ny}x{nz}_s{seed}", [parts, box], Params(r=r, xi=xi),
                    StepParams(dt=1.0 / 240.0, iters=10, steps=30),
                    meta=dict(n_particles=len(p)))


def c3(nx=100, ny=100, nz=200, seed=1003) -> Scene:
    """2,000,000 particles on a jittered 100x100x200 lattice filling the 1 x 1 x 2 m
    column, inside a closed static 1 x 1 x 2.2 m box of 12 inward triangles."""
    sx = 0.98 / (nx - 1)
    sz = 1.98 / (nz - 1)
    rng = np.random.Generator(np.random.PCG64(seed))
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1)
    p = g.reshape(-1, 3).astype(np.float64) * np.array([sx, sx, sz]) + 0.01
    p += rng.uniform(-1.5e-3, 1.5e-3, p.shape)
    parts = particles_mesh(p, 1.0 / PARTICLE_MASS)
    box = box_inward((0.0, 0.0, 0.0), (1.0, 1.0, 2.2))
    return assemble("c3", [parts, box], Params(r=5e-3, xi=5e-3),
                    StepParams(dt=1.0 / 240.0, iters=10, steps=30),
                    meta=dict(n_particles=len(p)))


def helix_strands(n_strands=16, seg=64, length=0.3, root_radius=0.2, center=(0.0, 0.0, 1.0),
                  curl=(2e-3, 10e-3), pitch=0.03, seed=1002, r=5e-4, xi=5e-4,
                  root_spacing_scale=1.0) -> Scene:
    """Strands rooted on a Fibonacci lattice over a sphere (roots pinned), each a
    helix about its outward radial axis.  The curl radius is ramped in from zero over
    the first 10 mm and clipped against the local strand spacing (times
    `root_spacing_scale`) so that neighbouring strands start well apart; a strand
    that still comes within 2r + xi of an earlier one has its curl radius halved
    until none does."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = seg + 1
    i = np.arange(n_strands) + 0.5
    phi = np.arccos(1 - 2 * i / n_strands)
    th = np.pi * (1 + 5 ** 0.5) * i
    dirs = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)
    roots = np.asarray(center) + root_radius * dirs
    # nearest-neighbour root distance
    d2 = ((roots[:, None, :] - roots[None, :, :]) ** 2).sum(-1) if n_strands <= 4096 else None
    if d2 is not None:
        np.fill_diagonal(d2, np.inf)
        dnn = np.sqrt(d2.min(1))
    else:
        dnn = np.full(n_strands, np.sqrt(4 * np.pi * root_radius ** 2 / n_strands))
    R = rng.uniform(curl[0], curl[1], n_strands)
    ph0 = rng.uniform(0, 2 * np.pi, n_strands)
    a = np.linspace(0.0, length, k)                         # axial distance from the root
    band = 2 * r + xi
    frames = []
    for s in range(n_strands):
        d = dirs[s]
        t1 = np.cross(d, [0.0, 0.0, 1.0] if abs(d[2]) < 0.9 else [1.0, 0.0, 0.0])
        t1 /= np.linalg.norm(t1)
        frames.append((d, t1, np.cross(d, t1)))

    def strand_points(s, radius):
        d, t1, t2 = frames[s]
        spacing = root_spacing_scale * dnn[s] * (root_radius + a) / root_radius
        rad = np.minimum(radius * np.clip(a / 0.01, 0.0, 1.0),
                         np.maximum(0.5 * spacing - band - 1e-4, 0.0))
        ang = ph0[s] + 2 * np.pi * a / pitch
        return roots[s] + a[:, None] * d + rad[:, None] * (np.cos(ang)[:, None] * t1 + np.sin(ang)[:, None] * t2)

    pts = np.empty((n_strands, k, 3))
    for s in range(n_strands):
        pts[s] = strand_points(s, R[s])
    # Strands that may still come within 2r + xi of another strand get their
    # curl radius halved, repeatedly.  The test samples segments and compares
    # sample points only, conservatively: two segments closer than `band` have
    # samples closer than band + delta, with delta the largest spacing of their
    # samples.  A coarse pass (4 samples per segment) finds the segment pairs of
    # different strands worth a look, a fine pass (32 per segment) decides.
    from scipy.spatial import cKDTree
    halvings = 0
    sub, fine = 4, 32
    tt = np.arange(sub) / sub
    tf = np.linspace(0.0, 1.0, fine + 1)
    for _ in range(40):
        dense = (pts[:, :-1, None, :] * (1 - tt)[None, None, :, None]
                 + pts[:, 1:, None, :] * tt[None, None, :, None]).reshape(n_strands, -1, 3)
        dense = np.concatenate([dense, pts[:, -1:, :]], 1)
        delta = float(np.max(np.linalg.norm(np.diff(dense, axis=1), axis=2)))
        per = dense.shape[1]
        close = cKDTree(dense.reshape(-1, 3)).query_pairs(band + delta, output_type="ndarray")
        sa, sb = close[:, 0] // per, close[:, 1] // per
        cross = sa != sb
        ga = np.minimum((close[cross, 0] % per) // sub, k - 2)
        gb = np.minimum((close[cross, 1] % per) // sub, k - 2)
        cand = np.unique(np.stack([sa[cross], ga, sb[cross], gb], 1), axis=0)
        flagged = []
        for c in range(0, len(cand), 256):
            q = cand[c:c + 256]
            A = pts[q[:, 0], q[:, 1]][:, None, :] * (1 - tf)[None, :, None] + \
                pts[q[:, 0], q[:, 1] + 1][:, None, :] * tf[None, :, None]
            B = pts[q[:, 2], q[:, 3]][:, None, :] * (1 - tf)[None, :, None] + \
                pts[q[:, 2], q[:, 3] + 1][:, None, :] * tf[None, :, None]
            dmin = np.sqrt(((A[:, :, None, :] - B[:, None, :, :]) ** 2).sum(-1).min((1, 2)))
            step = np.maximum(np.linalg.norm(A[:, 1] - A[:, 0], axis=1), np.linalg.norm(B[:, 1] - B[:, 0], axis=1))
            flagged.append(q[dmin < band + step])
        flagged = np.concatenate(flagged, 0) if flagged else np.zeros((0, 4), np.int64)
        if not len(flagged):
            break
        # of each close pair of strands the later one is halved (the earlier is
        # accepted), unless its curl is already negligible: then the earlier one
        lo_s, hi_s = np.minimum(flagged[:, 0], flagged[:, 2]), np.maximum(flagged[:, 0], flagged[:, 2])
        halve = np.unique(np.where(R[hi_s] > 1e-4, hi_s, lo_s))
        halvings += len(halve)
        R[halve] *= 0.5
        for s in halve.tolist():
            pts[s] = strand_points(s, R[s])
    w = np.full((n_strands, k), 1.0 / STRAND_VERTEX_MASS)
    w[:, 0] = 0.0
    m = strands_mesh(pts, w)
    return assemble(f"strands{n_strands}x{seg}_s{seed}", [m], Params(r=r, xi=xi),
                    StepParams(dt=1.0 / 240.0, iters=10, steps=30),
                    meta=dict(n_strands=n_strands, seg=seg, curl_halvings=halvings))


def strand_bundle(nx=3, ny=3, seg=16, spacing=1.2e-3, seg_len=4.69e-3, wiggle=1e-4, seed=21,
                  r=5e-4, xi=5e-4) -> Scene:
    """Hanging strands on an nx x ny lattice `spacing` apart (inside the contact
    band 2r + xi for the defaults), roots pinned at z = 1, each with a small
    seeded sinusoidal wiggle: dense edge-edge pairs between neighbours."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = seg + 1
    pts = np.empty((nx * ny, k, 3))
    z = 1.0 - seg_len * np.arange(k)
    for s in range(nx * ny):
        i, j = divmod(s, ny)
        ph = rng.uniform(0, 2 * np.pi, 2)
        amp = wiggle * np.clip(np.arange(k) / 3.0, 0, 1)
        pts[s, :, 0] = i * spacing + amp * np.sin(0.9 * np.arange(k) + ph[0])
        pts[s, :, 1] = j * spacing + amp * np.cos(0.7 * np.arange(k) + ph[1])
        pts[s, :, 2] = z
    w = np.full((nx * ny, k), 1.0 / STRAND_VERTEX_MASS)
    w[:, 0] = 0.0
    return assemble(f"bundle{nx}x{ny}x{seg}_s{seed}", [strands_mesh(pts, w)], Params(r=r, xi=xi),
                    StepParams(dt=1.0 / 240.0, iters=10, steps=30),
                    meta=dict(n_strands=nx * ny, seg=seg))


def c2(seed=1002) -> Scene:
    """10,000 pinned-root helical strands of 64 segments (650,000 vertices)."""
    sc = helix_strands(n_strands=10000, seg=64, seed=seed)
    sc.name = "c2"
    return sc


def rod_lattice(n_per_layer=16, seg=60, length=30.0, pitch=2.0, z0=1.0, dz=0.15, inv_mass=50.0) -> _Mesh:
    """Two crossing layers of straight rods (a wire structure): n_per_layer rods
    along x at height z0, n_per_layer along y at z0 + dz, each of `seg`
    segments spanning `length`, `pitch` apart, both ends pinned."""
    k = seg + 1
    t = np.linspace(-0.5 * length, 0.5 * length, k)
    off = (np.arange(n_per_layer) - 0.5 * (n_per_layer - 1)) * pitch
    pts = np.empty((2 * n_per_layer, k, 3))
    for r, o in enumerate(off):
        pts[r, :, 0], pts[r, :, 1], pts[r, :, 2] = t, o, z0
        pts[n_per_layer + r, :, 0], pts[n_per_layer + r, :, 1], pts[n_per_layer + r, :, 2] = o, t, z0 + dz
    w = np.full((2 * n_per_layer, k), inv_mass)
    w[:, 0] = w[:, -1] = 0.0
    return strands_mesh(pts, w)


def octopus(center, radius=3.0, level=3, arms=8, arm_seg=12, arm_len=0.4, arm_z=1.35, phase=0.0,
            inv_mass=20.0) -> _Mesh:
    """A deformable closed surface with strand arms (a synthetic stand-in for a
    tentacled soft body): a dynamic icosphere and `arms` polylines, each
    attached to the sphere vertex nearest its root direction on the lower
    hemisphere and running radially outwards, dropping to height arm_z."""
    body = icosphere(level, radius, center)
    c = np.asarray(center, np.float64)
    xs = [body.x]
    edges = []
    n0 = len(body.x)
    for a in range(arms):
        th = phase + 2.0 * np.pi * a / arms
        d = np.array([math.cos(th), math.sin(th)])
        root_dir = np.array([0.5 * d[0], 0.5 * d[1], -math.sqrt(0.75)])   # 30 degrees from the bottom
        root = int(np.argmax((body.x - c) @ root_dir))
        r0 = body.x[root]
        rh = float(np.hypot(*(r0[:2] - c[:2])))
        pts = np.empty((arm_seg, 3))
        for j in range(1, arm_seg + 1):
            h = rh + arm_len * j
            pts[j - 1, :2] = c[:2] + h * d
            pts[j - 1, 2] = max(arm_z, r0[2] - arm_len * j)
        first = n0 + sum(len(q) for q in xs[1:])
        edges.append([root, first])
        edges += [[first + j, first + j + 1] for j in range(arm_seg - 1)]
        xs.append(pts)
    m = _Mesh(np.concatenate(xs, 0), body.tris, np.full(n0 + arms * arm_seg, inv_mass))
    m.extra_edges = np.asarray(edges, np.int64)
    return m


def c5(seed=1005, n_rods=16, rod_seg=60, side=95.0, body_level=3, body_radius=9.0, arm_seg=12, arm_len=1.2,
       n_paper=64, part=(39, 39, 4), part_spacing=0.8, name="c5") -> Scene:
    """Coupled codimensional scene: a floor, a pinned two-layer rod lattice
    (2 x n_rods rods of rod_seg segments spanning `side`), two soft tentacled
    bodies resting on it, a paper sheet over their tops and a block of free
    particles (`part` = nx x ny x nz, `part_spacing` apart) over the sheet's
    centre; each layer lies 0.15 (the particles 0.2) above the one below,
    inside the interaction range 2r + xi = 0.86 (13,612 vertices at the
    defaults; rod, arm and sheet segments about 1.5 long).  Lengths are in the
    units of the contact parameters r = 0.4, xi = 0.06, delta = 0.01; the
    paper sheet and the particles start with small random velocities."""
    rng = np.random.Generator(np.random.PCG64(seed))
    floor = ground_quad(2.0 * side, 0.0)
    pitch = side / (n_rods - 0.5)
    rods = rod_lattice(n_per_layer=n_rods, seg=rod_seg, length=side, pitch=pitch)
    top_rods = 1.15
    gap = 0.15
    R = body_radius
    zc = top_rods + gap + R
    octo = [octopus((-0.27 * side, -0.1 * side, zc), radius=R, level=body_level, arm_seg=arm_seg, arm_len=arm_len,
                    phase=0.0),
            octopus((0.27 * side, 0.1 * side, zc), radius=R, level=body_level, arm_seg=arm_seg, arm_len=arm_len,
                    phase=np.pi / 8)]
    z_paper = zc + R + gap
    paper = cloth_grid(n_paper, side, (0.0, 0.0, z_paper))
    paper.inv_mass = np.full(len(paper.x), 100.0)
    paper.v = rng.normal(0.0, 0.3, paper.x.shape)
    nx, ny, nz = part
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1).reshape(-1, 3)
    p = (g - np.array([0.5 * (nx - 1), 0.5 * (ny - 1), 0.0])) * part_spacing
    p[:, 2] += z_paper + 0.2
    p += rng.uniform(-0.03, 0.03, p.shape)
    parts = particles_mesh(p, 80.0)
    parts.v = rng.normal(0.0, 0.3, parts.x.shape)
    return assemble(name, [floor, rods] + octo + [paper, parts], Params(r=0.4, xi=0.06, delta=0.01),
                    StepParams(dt=1.0 / 120.0, iters=10, steps=30),
                    meta=dict(n_particles=len(p), n_paper=n_paper * n_paper))


def c5_small(seed=1006) -> Scene:
    """The coupled scene at a size the oracle steps in a fraction of a second:
    2 x 4 rods of 20 segments over 30 units, two bodies of radius 4.5
    (162-vertex spheres, arms of 5 segments), a 21 x 21 paper sheet and an
    8 x 8 x 3 particle block."""
    return c5(seed=seed, n_rods=4, rod_seg=20, side=30.0, body_level=2, body_radius=4.5, arm_seg=5,
              n_paper=21, part=(8, 8, 3), name="c5_small")


# --------------------------------------------------------------------------
# the batched / served workload
# --------------------------------------------------------------------------

@dataclass
class Request:
    rid: int
    arrival: float      # seconds after the stream starts
    scene: Scene


def c4_requests(n_requests=512, rate=200.0, seed=4999, lo=16, hi=512, steps=30) -> list:
    """Poisson stream of independent drape-on-sphere requests whose cloth side (in
    vertices) is log-uniform in [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    out = []
    for i in range(n_requests):
        rr = np.random.Generator(np.random.PCG64(4000 + i))
        n = int(round(math.exp(rr.uniform(math.log(lo), math.log(hi)))))
        h = 1.0 / (n - 1)
        rad = min(2e-3, h / 4)
        off = rr.uniform(-0.25, 0.25, 2)
        rot = rr.uniform(0, 2 * np.pi)
        jit = np.array([0.0, 0.0, min(1e-3, h / 8)])
        sc = drape(n=n, side=1.0, jitter=jit, seed=4000 + i, r=rad, xi=rad,
                   offset_xy=tuple(off), rot=rot, steps=steps, name=f"req{i}_n{n}")
        out.append(Request(i, float(t[i]), sc))
    return out


SCENES = {
    "c0": c0,
    "c1": c1,
    "c2": c2,
    "c3": c3,
    "c5": c5,
}
