"""ctypes front end of the FP64 CPU oracle (oracle/libccfr_oracle.so).

TEST INFRASTRUCTURE ONLY: a plain, slow, literal implementation of the CCFR hot
path written from the paper (Kikuchi & Kanai, "Convex Collision-Free Regions",
Eq. 1-3 and Algorithms 1-4).  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it.  It shares no code with the HIP
library in paper_2607_26901_amd/.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libccfr_oracle.so")

KIND_VE, KIND_VF, KIND_EE, KIND_VV = 0, 1, 2, 3

HS_DTYPE = np.dtype([("n", "<f8", (3,)), ("d", "<f8"), ("phi", "<f8"), ("share", "<f8"), ("key", "<u8"),
                     ("fragile", "<i4"), ("pad", "<i4")])
assert HS_DTYPE.itemsize == 64


class OrcParams(C.Structure):
    _fields_ = [("r", C.c_double), ("xi", C.c_double), ("delta", C.c_double), ("guard", C.c_double),
                ("eps_retract", C.c_double), ("eps_plesnik", C.c_double),
                ("max_passes", C.c_int32), ("response", C.c_int32), ("resp_compliance", C.c_double),
                ("vis_width", C.c_double), ("mu_s", C.c_double), ("mu_k", C.c_double)]


class OrcMesh(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("n_tris", C.c_int32), ("n_edges", C.c_int32),
                ("pad_", C.c_int32), ("x", C.c_void_p), ("inv_mass", C.c_void_p),
                ("tris", C.c_void_p), ("edges", C.c_void_p)]


class OrcStepParams(C.Structure):
    _fields_ = [("dt", C.c_double), ("g", C.c_double * 3), ("iters", C.c_int32),
                ("n_colors", C.c_int32), ("alpha", C.c_double), ("early_exit", C.c_int32),
                ("pad_", C.c_int32), ("conv_tol", C.c_double)]


_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        lib = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        lib.orc_box_pad.restype = C.c_float
        lib.orc_box_pad.argtypes = [vp]
        lib.orc_candidates.argtypes = [vp, vp, vp, i64, vp, i64, vp, i64, vp, i64, vp]
        for f in ("orc_vf_tris_of_vertex", "orc_vf_verts_of_tri", "orc_ee_partners_of_edge",
                  "orc_vv_partners_of_vertex", "orc_ve_edges_of_vertex", "orc_ve_verts_of_edge"):
            getattr(lib, f).restype = i64
            getattr(lib, f).argtypes = [vp, vp, i32, vp, i64]
        lib.orc_regions.restype = i64
        lib.orc_regions.argtypes = [vp, vp, vp, i64, vp, i64, vp, i64, vp, i64, vp, vp, i64, vp]
        lib.orc_vertex_region.restype = i64
        lib.orc_vertex_region.argtypes = [vp, vp, i32, vp, i64]
        lib.orc_project.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.orc_project_one.restype = C.c_int
        lib.orc_project_one.argtypes = [vp, dbl, vp, vp, i64, vp, vp, vp]
        lib.orc_project_branches.restype = C.c_int
        lib.orc_project_branches.argtypes = [vp, dbl, vp, vp, i64, vp, vp, vp, C.c_int, vp]
        lib.orc_apply_response.argtypes = [vp, dbl, vp, i64, dbl, vp, vp]
        lib.orc_response.argtypes = [vp, vp, vp, vp, dbl, vp, vp]
        lib.orc_orthogonal_projection.argtypes = [vp, vp, vp, dbl, vp, dbl]
        lib.orc_closest_point_triangle.restype = C.c_int
        lib.orc_closest_point_triangle.argtypes = [vp] * 6
        lib.orc_closest_points_segments.restype = C.c_int
        lib.orc_closest_points_segments.argtypes = [vp] * 6
        lib.orc_color_edges.restype = i32
        lib.orc_color_edges.argtypes = [i32, i32, vp, vp]
        lib.orc_xpbd_step.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp]
        lib.orc_count_edge_tri_intersections.restype = i64
        lib.orc_count_edge_tri_intersections.argtypes = [i32, vp, i32, vp, i32, vp]
        lib.orc_min_separation.restype = dbl
        lib.orc_min_separation.argtypes = [i32, vp, vp, i32, vp, i32, vp, dbl, dbl, vp]
        lib.orc_min_separation_grid.restype = dbl
        lib.orc_min_separation_grid.argtypes = [i32, vp, vp, i32, vp, i32, vp, dbl, dbl, vp]
        lib.orc_motion_check.restype = dbl
        lib.orc_motion_check.argtypes = [i32, vp, vp, vp, i32, vp, i32, vp, dbl, dbl, i64, vp, vp, vp]
        lib.orc_orient3d_sign.restype = C.c_int
        lib.orc_orient3d_sign.argtypes = [vp] * 4
        lib.orc_orient2d_sign.restype = C.c_int
        lib.orc_orient2d_sign.argtypes = [vp] * 3
        lib.orc_num_threads.restype = C.c_int
        lib.orc_set_num_threads.argtypes = [C.c_int]
        lib.orc_fragile_reasons.argtypes = [vp, C.c_int]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def params(p) -> OrcParams:
    """From a scenes.Params (its float values are used as given)."""
    f = lambda v: float(np.float32(v))  # the GPU path receives these as FP32
    g = lambda name, default=0.0: f(getattr(p, name, default))
    return OrcParams(f(p.r), f(p.xi), f(p.delta), f(p.guard), f(p.eps_retract), f(p.eps_plesnik),
                     int(p.max_passes), int(bool(getattr(p, "response", False))), g("resp_compliance"),
                     g("vis_width"), g("mu_s"), g("mu_k"))


class Mesh:
    """Keeps FP64 copies of a scene's arrays alive for the C side."""

    def __init__(self, scene, x=None):
        self.x = np.ascontiguousarray(scene.x if x is None else x, np.float64).reshape(-1, 3)
        self.inv_mass = np.ascontiguousarray(scene.inv_mass, np.float64)
        self.tris = np.ascontiguousarray(scene.tris, np.int32).reshape(-1, 3)
        self.edges = np.ascontiguousarray(scene.edges, np.int32).reshape(-1, 2)
        self.c = OrcMesh(len(self.x), len(self.tris), len(self.edges), 0, _p(self.x).value,
                         _p(self.inv_mass).value, _p(self.tris).value, _p(self.edges).value)

    @property
    def ref(self):
        return C.byref(self.c)


def box_pad(p) -> np.float32:
    return np.float32(load().orc_box_pad(C.byref(params(p))))


def candidates(mesh: Mesh, p) -> dict:
    lib = load()
    prm = params(p)
    counts = np.zeros(4, np.int64)
    n = len(mesh.x)
    caps = [8 * n + 64, 8 * len(mesh.edges) + 64, 8 * n + 64, 8 * n + 64]
    while True:
        bufs = [np.zeros((c, 2), np.int32) for c in caps]
        lib.orc_candidates(mesh.ref, C.byref(prm), _p(bufs[0]), caps[0], _p(bufs[1]), caps[1],
                           _p(bufs[2]), caps[2], _p(bufs[3]), caps[3], _p(counts))
        if all(counts[k] <= caps[k] for k in range(4)):
            return {"vf": bufs[0][:counts[0]].copy(), "ee": bufs[1][:counts[1]].copy(),
                    "vv": bufs[2][:counts[2]].copy(), "ve": bufs[3][:counts[3]].copy()}
        caps = [int(max(counts[k], caps[k])) for k in range(4)]


def _partners(fn, mesh, p, idx) -> np.ndarray:
    prm = params(p)
    cap = 256
    while True:
        out = np.zeros(cap, np.int32)
        n = fn(mesh.ref, C.byref(prm), int(idx), _p(out), cap)
        if n <= cap:
            return out[:n].copy()
        cap = int(n)


def vf_tris_of_vertex(mesh, p, v):
    return _partners(load().orc_vf_tris_of_vertex, mesh, p, v)


def vf_verts_of_tri(mesh, p, t):
    return _partners(load().orc_vf_verts_of_tri, mesh, p, t)


def ee_partners_of_edge(mesh, p, e):
    return _partners(load().orc_ee_partners_of_edge, mesh, p, e)


def vv_partners_of_vertex(mesh, p, v):
    return _partners(load().orc_vv_partners_of_vertex, mesh, p, v)


def ve_edges_of_vertex(mesh, p, v):
    return _partners(load().orc_ve_edges_of_vertex, mesh, p, v)


def ve_verts_of_edge(mesh, p, e):
    return _partners(load().orc_ve_verts_of_edge, mesh, p, e)


def regions(mesh: Mesh, p, cands: dict):
    """Returns (offsets [N+1] int64, half-spaces [H] HS_DTYPE, n_degenerate)."""
    lib = load()
    prm = params(p)
    vf = np.ascontiguousarray(cands["vf"], np.int32)
    ee = np.ascontiguousarray(cands["ee"], np.int32)
    vv = np.ascontiguousarray(cands["vv"], np.int32)
    ve = np.ascontiguousarray(cands.get("ve", np.zeros((0, 2))), np.int32).reshape(-1, 2)
    n = len(mesh.x)
    offsets = np.zeros(n + 1, np.int64)
    stats = np.zeros(4, np.int64)
    H = lib.orc_regions(mesh.ref, C.byref(prm), _p(vf), len(vf), _p(ee), len(ee), _p(vv), len(vv),
                        _p(ve), len(ve), _p(offsets), None, 0, _p(stats))
    hs = np.zeros(max(H, 1), HS_DTYPE)
    lib.orc_regions(mesh.ref, C.byref(prm), _p(vf), len(vf), _p(ee), len(ee), _p(vv), len(vv),
                    _p(ve), len(ve), _p(offsets), _p(hs), H, _p(stats))
    return offsets, hs[:H], int(stats[0])


def vertex_region(mesh: Mesh, p, v: int) -> np.ndarray:
    lib = load()
    prm = params(p)
    cap = 256
    while True:
        hs = np.zeros(cap, HS_DTYPE)
        n = lib.orc_vertex_region(mesh.ref, C.byref(prm), int(v), _p(hs), cap)
        if n <= cap:
            return hs[:n].copy()
        cap = int(n)


def project(mesh: Mesh, p, offsets, hs, y):
    """Alg. 2 + Alg. 1 + r-clamp per vertex.  Returns (y_out, halted, fragile, stats)."""
    lib = load()
    prm = params(p)
    offsets = np.ascontiguousarray(offsets, np.int64)
    hs = np.ascontiguousarray(hs, HS_DTYPE)
    if len(hs) == 0:
        hs = np.zeros(1, HS_DTYPE)
    y = np.ascontiguousarray(y, np.float64).reshape(-1, 3)
    out = np.zeros_like(y)
    halted = np.zeros(len(y), np.int8)
    fragile = np.zeros(len(y), np.int8)
    stats = np.zeros(4, np.int64)
    lib.orc_project(mesh.ref, C.byref(prm), _p(offsets), _p(hs), _p(y), _p(out), _p(halted),
                    _p(fragile), _p(stats))
    return out, halted, fragile, stats


def project_one(p, inv_mass, x, hs, y):
    """Returns (y_out, halted, fragile) for one vertex."""
    lib = load()
    prm = params(p)
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    hs = np.ascontiguousarray(hs, HS_DTYPE)
    if len(hs) == 0:
        hs1 = np.zeros(1, HS_DTYPE)
    else:
        hs1 = hs
    out = np.zeros(3)
    frag = C.c_int(0)
    h = lib.orc_project_one(C.byref(prm), float(inv_mass), _p(x), _p(hs1), len(hs), _p(y), _p(out),
                            C.byref(frag))
    return out, int(h), int(frag.value)


def project_branches(p, inv_mass, x, hs, y, cap=256):
    """Every result of Alg. 2 for one vertex over the branches of its
    near-threshold decisions.  Returns (y_outs [k][3], halts [k], complete)."""
    lib = load()
    prm = params(p)
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    hs = np.ascontiguousarray(hs, HS_DTYPE)
    hs1 = hs if len(hs) else np.zeros(1, HS_DTYPE)
    outs = np.zeros((cap, 3))
    halts = np.zeros(cap, np.int8)
    comp = C.c_int(0)
    n = lib.orc_project_branches(C.byref(prm), float(inv_mass), _p(x), _p(hs1), len(hs), _p(y), _p(outs),
                                 _p(halts), int(cap), C.byref(comp))
    return outs[:n].copy(), halts[:n].copy(), bool(comp.value)


def apply_response(p, inv_mass, hs, dt, y):
    """applyResponse (Sec. 3.3) for one vertex: the displacement after the
    response and friction of its active contacts."""
    prm = params(p)
    hs = np.ascontiguousarray(hs, HS_DTYPE)
    hs1 = hs if len(hs) else np.zeros(1, HS_DTYPE)
    y = np.ascontiguousarray(y, np.float64)
    out = np.zeros(3)
    load().orc_apply_response(C.byref(prm), float(inv_mass), _p(hs1), len(hs), float(dt), _p(y), _p(out))
    return out


def response(mesh: "Mesh", p, offsets, hs, dt, y):
    """applyResponse for every vertex of a mesh."""
    prm = params(p)
    offsets = np.ascontiguousarray(offsets, np.int64)
    hs = np.ascontiguousarray(hs, HS_DTYPE)
    hs1 = hs if len(hs) else np.zeros(1, HS_DTYPE)
    y = np.ascontiguousarray(y, np.float64).reshape(-1, 3)
    out = np.zeros_like(y)
    load().orc_response(mesh.ref, C.byref(prm), _p(offsets), _p(hs1), float(dt), _p(y), _p(out))
    return out


def make_halfspaces(n, d, keys=None, phi=None, share=None) -> np.ndarray:
    n = np.asarray(n, np.float64).reshape(-1, 3)
    hs = np.zeros(len(n), HS_DTYPE)
    hs["n"] = n
    hs["d"] = np.asarray(d, np.float64).reshape(-1)
    hs["phi"] = hs["d"] if phi is None else phi
    hs["share"] = 1.0 if share is None else share
    hs["key"] = np.arange(len(n), dtype=np.uint64) if keys is None else np.asarray(keys, np.uint64)
    return hs


class EroState:
    """Alg. 1 state {m, V, A, B} for driving orthogonalProjection directly."""

    def __init__(self):
        self.buf = np.zeros(22)

    @property
    def m(self):
        return int(self.buf[0])


def orthogonal_projection(xt, x0, n, b, state: EroState, eps=1e-6):
    xt = np.ascontiguousarray(xt, np.float64).copy()
    x0 = np.ascontiguousarray(x0, np.float64)
    n = np.ascontiguousarray(n, np.float64)
    load().orc_orthogonal_projection(_p(xt), _p(x0), _p(n), float(b), _p(state.buf), float(eps))
    return xt


def closest_point_triangle(p, a, b, c):
    q = np.zeros(3)
    bary = np.zeros(3)
    arr = [np.ascontiguousarray(v, np.float64) for v in (p, a, b, c)]
    rc = load().orc_closest_point_triangle(*[_p(v) for v in arr], _p(q), _p(bary))
    return rc, q, bary


def closest_points_segments(a, b, c, d):
    s = C.c_double(0)
    t = C.c_double(0)
    arr = [np.ascontiguousarray(v, np.float64) for v in (a, b, c, d)]
    rc = load().orc_closest_points_segments(*[_p(v) for v in arr], C.byref(s), C.byref(t))
    return rc, s.value, t.value


def color_edges(n_verts, edges) -> tuple:
    edges = np.ascontiguousarray(edges, np.int32)
    col = np.zeros(max(len(edges), 1), np.int32)
    nc = load().orc_color_edges(int(n_verts), len(edges), _p(edges), _p(col))
    return col[:len(edges)], int(nc)


class Sim:
    """FP64 state of one scene stepped by the oracle's Alg. 4."""

    def __init__(self, scene, x=None, v=None):
        self.scene = scene
        self.x = np.ascontiguousarray(scene.x if x is None else x, np.float64).copy()
        self.v = np.ascontiguousarray(scene.v if v is None else v, np.float64).copy()
        self.w = np.ascontiguousarray(scene.inv_mass, np.float64)
        self.tris = np.ascontiguousarray(scene.tris, np.int32)
        self.edges = np.ascontiguousarray(scene.edges, np.int32)
        rx = scene.rest_x.astype(np.float64)
        self.rest = np.linalg.norm(rx[self.edges[:, 0]] - rx[self.edges[:, 1]], axis=1) \
            if len(self.edges) else np.zeros(1)
        self.color, self.n_colors = color_edges(len(self.x), self.edges)
        self.counters = np.zeros(12, np.int64)

    def step(self, iters=None, trace=False):
        """One substep; with trace=True returns the anchor after every iteration
        ([iters][N][3])."""
        sp = self.scene.step
        osp = OrcStepParams(float(np.float32(sp.dt)), (C.c_double * 3)(*[float(np.float32(g)) for g in sp.gravity]),
                            int(sp.iters if iters is None else iters), self.n_colors,
                            float(np.float32(sp.alpha)), int(bool(getattr(sp, "early_exit", False))), 0,
                            float(np.float32(getattr(sp, "conv_tol", 0.0))))
        prm = params(self.scene.params)
        tr = np.zeros((osp.iters, len(self.x), 3)) if trace else None
        load().orc_xpbd_step(len(self.x), len(self.tris), len(self.edges), _p(self.tris),
                             _p(self.edges), _p(self.w), _p(self.rest),
                             _p(self.color if len(self.color) else np.zeros(1, np.int32)),
                             self.n_colors, _p(self.x), _p(self.v), C.byref(prm), C.byref(osp),
                             _p(self.counters), None if tr is None else _p(tr))
        return tr


def count_intersections(x, tris, edges) -> int:
    x = np.ascontiguousarray(x, np.float64)
    tris = np.ascontiguousarray(tris, np.int32)
    edges = np.ascontiguousarray(edges, np.int32)
    return int(load().orc_count_edge_tri_intersections(len(x), _p(x), len(tris), _p(tris),
                                                       len(edges), _p(edges)))


def min_separation(x, inv_mass, tris, edges, reach, below):
    """Returns (min distance (capped at reach), counts below [VF, EE, VV, VE])."""
    x = np.ascontiguousarray(x, np.float64)
    w = np.ascontiguousarray(inv_mass, np.float64)
    tris = np.ascontiguousarray(tris, np.int32)
    edges = np.ascontiguousarray(edges, np.int32)
    cnt = np.zeros(4, np.int64)
    d = load().orc_min_separation(len(x), _p(x), _p(w), len(tris), _p(tris), len(edges), _p(edges),
                                  float(reach), float(below), _p(cnt))
    return float(d), cnt


def min_separation_grid(x, inv_mass, tris, edges, reach, below):
    """min_separation through a uniform grid, for large meshes."""
    x = np.ascontiguousarray(x, np.float64)
    w = np.ascontiguousarray(inv_mass, np.float64)
    tris = np.ascontiguousarray(tris, np.int32)
    edges = np.ascontiguousarray(edges, np.int32)
    cnt = np.zeros(4, np.int64)
    d = load().orc_min_separation_grid(len(x), _p(x), _p(w), len(tris), _p(tris), len(edges), _p(edges),
                                       float(reach), float(below), _p(cnt))
    return float(d), cnt


def motion_check(x0, x1, inv_mass, tris, edges, floor, reach, max_samples=10000):
    """Certified sampled check of the straight-line motion x0 -> x1.  Returns
    (smallest sampled distance, certified, samples, t of the smallest)."""
    x0 = np.ascontiguousarray(x0, np.float64)
    x1 = np.ascontiguousarray(x1, np.float64)
    w = np.ascontiguousarray(inv_mass, np.float64)
    tris = np.ascontiguousarray(tris, np.int32)
    edges = np.ascontiguousarray(edges, np.int32)
    cert = C.c_int32(0)
    ns = C.c_int64(0)
    tm = C.c_double(0)
    d = load().orc_motion_check(len(x0), _p(x0), _p(x1), _p(w), len(tris), _p(tris), len(edges), _p(edges),
                                float(floor), float(reach), int(max_samples), C.byref(cert), C.byref(ns),
                                C.byref(tm))
    return float(d), bool(cert.value), int(ns.value), float(tm.value)


def orient3d_sign(a, b, c, d) -> int:
    arr = [np.ascontiguousarray(v, np.float64) for v in (a, b, c, d)]
    return int(load().orc_orient3d_sign(*[_p(v) for v in arr]))


def orient2d_sign(a, b, c) -> int:
    arr = [np.ascontiguousarray(v, np.float64) for v in (a, b, c)]
    return int(load().orc_orient2d_sign(*[_p(v) for v in arr]))


def num_threads() -> int:
    return int(load().orc_num_threads())


def set_num_threads(n: int) -> None:
    load().orc_set_num_threads(int(n))


def fragile_reasons(reset=True) -> np.ndarray:
    out = np.zeros(3, np.int64)
    load().orc_fragile_reasons(_p(out), int(reset))
    return out
