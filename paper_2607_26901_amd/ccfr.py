"""Python binding of the gfx950 CCFR library (libccfr.so, C ABI in include/ccfr.h).

Argument marshalling only: every step of the hot path runs in the library's HIP
kernels.  Device arrays are torch tensors on the GPU (contiguous float32 /
int32), which supply memory; calls are enqueued on torch's current stream.
Importing this module does not touch the GPU; loading the library fails loudly
when it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libccfr.so")

HALFSPACE_DTYPE = np.dtype([("n", "<f4", (3,)), ("d", "<f4"), ("phi", "<f4"), ("share", "<f4"),
                            ("key", "<u8")])
assert HALFSPACE_DTYPE.itemsize == 32

STATUS_NAMES = {0: "ok", -1: "invalid argument", -2: "capacity", -3: "hip", -4: "non-finite",
                -5: "degenerate", -6: "not ready", -7: "no memory"}


class CcfrError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)} ({code})")
        self.code = code


FLAG_RESPONSE = 1


class Params(C.Structure):
    _fields_ = [("r", C.c_float), ("xi", C.c_float), ("delta", C.c_float), ("guard", C.c_float),
                ("eps_retract", C.c_float), ("eps_plesnik", C.c_float), ("max_passes", C.c_int32),
                ("flags", C.c_int32), ("resp_compliance", C.c_float), ("vis_width", C.c_float),
                ("mu_s", C.c_float), ("mu_k", C.c_float)]


class Candidates(C.Structure):
    _fields_ = [("vf", C.c_void_p), ("ee", C.c_void_p), ("vv", C.c_void_p), ("counts_dev", C.c_void_p),
                ("cap_vf", C.c_int64), ("cap_ee", C.c_int64), ("cap_vv", C.c_int64), ("ve", C.c_void_p),
                ("cap_ve", C.c_int64)]


class Regions(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("pad_", C.c_int32), ("offsets", C.c_void_p), ("hs", C.c_void_p),
                ("cap", C.c_int64)]


class StepParams(C.Structure):
    _fields_ = [("dt", C.c_float), ("gravity", C.c_float * 3), ("iters", C.c_int32), ("alpha", C.c_float),
                ("collision", Params), ("early_exit", C.c_int32), ("conv_tol", C.c_float)]


class Tuning(C.Structure):
    _fields_ = [("cell_scale", C.c_float), ("pair_split", C.c_int32), ("pair_reuse", C.c_int32),
                ("pair_skin", C.c_int32), ("broad_phase", C.c_int32), ("direct_regions", C.c_int32)]


class StatusInfo(C.Structure):
    _fields_ = [("status_bits", C.c_uint32), ("last_counts", C.c_int32 * 3), ("last_contacts", C.c_int32),
                ("last_halfspaces", C.c_int32), ("need", C.c_int64 * 6), ("totals", C.c_int64 * 10),
                ("candidate_builds", C.c_int64), ("iterations_run", C.c_int64), ("halt_runs", C.c_int64 * 2),
                ("max_halt_run", C.c_int32), ("last_ve", C.c_int32), ("need_ve", C.c_int64),
                ("total_ve", C.c_int64)]


EXPORTS = ["ccfr_status_string", "ccfr_create", "ccfr_destroy", "ccfr_mesh_create", "ccfr_mesh_destroy",
           "ccfr_mesh_edges", "ccfr_mesh_inv_mass_dev", "ccfr_reserve", "ccfr_build_candidates",
           "ccfr_build_regions", "ccfr_project_displacements", "ccfr_project_displacements_noalloc",
           "ccfr_apply_response",
           "ccfr_xpbd_step", "ccfr_xpbd_step_traced",
           "ccfr_sync_status",
           "ccfr_profile_enable", "ccfr_profile_read", "ccfr_set_tuning", "ccfr_get_tuning",
           "ccfr_batch_create", "ccfr_batch_destroy", "ccfr_batch_footprint", "ccfr_batch_add",
           "ccfr_batch_remove", "ccfr_batch_step", "ccfr_batch_rollback", "ccfr_batch_read", "ccfr_batch_stats"]

_lib = None


def load():
    """Load libccfr.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2607_26901_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    lib.ccfr_status_string.restype = C.c_char_p
    lib.ccfr_status_string.argtypes = [C.c_int]
    lib.ccfr_create.argtypes = [C.POINTER(vp), C.c_int]
    lib.ccfr_destroy.argtypes = [vp]
    lib.ccfr_destroy.restype = None
    lib.ccfr_mesh_create.argtypes = [vp, i32, vp, i32, vp, i32, vp, vp, C.POINTER(vp)]
    lib.ccfr_mesh_destroy.argtypes = [vp]
    lib.ccfr_mesh_destroy.restype = None
    lib.ccfr_mesh_edges.argtypes = [vp, C.POINTER(i32), vp]
    lib.ccfr_mesh_inv_mass_dev.restype = vp
    lib.ccfr_mesh_inv_mass_dev.argtypes = [vp]
    lib.ccfr_reserve.argtypes = [vp, i64, i64, i64, i64, i64, i64, vp]
    lib.ccfr_build_candidates.argtypes = [vp, vp, vp, C.POINTER(Params), C.POINTER(Candidates), vp]
    lib.ccfr_build_regions.argtypes = [vp, vp, vp, C.POINTER(Candidates), C.POINTER(Params),
                                       C.POINTER(Regions), vp]
    lib.ccfr_project_displacements.argtypes = [vp, C.POINTER(Regions), vp, vp, C.POINTER(Params), vp, vp, vp]
    lib.ccfr_project_displacements_noalloc.argtypes = [C.POINTER(Regions), vp, vp, C.POINTER(Params), vp, vp,
                                                       vp, vp]
    lib.ccfr_apply_response.argtypes = [vp, C.POINTER(Regions), vp, vp, C.POINTER(Params), C.c_float, vp, vp]
    lib.ccfr_xpbd_step.argtypes = [vp, vp, vp, vp, C.POINTER(StepParams), vp]
    lib.ccfr_xpbd_step_traced.argtypes = [vp, vp, vp, vp, C.POINTER(StepParams), vp, vp]
    lib.ccfr_sync_status.argtypes = [vp, vp, C.POINTER(StatusInfo), C.c_int]
    lib.ccfr_profile_enable.argtypes = [vp, C.c_int]
    lib.ccfr_profile_read.argtypes = [vp, vp, vp, vp]
    lib.ccfr_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
    lib.ccfr_get_tuning.argtypes = [vp, C.POINTER(Tuning)]
    lib.ccfr_batch_create.argtypes = [vp, i32, i64, i64, i64, C.POINTER(vp)]
    lib.ccfr_batch_destroy.argtypes = [vp]
    lib.ccfr_batch_destroy.restype = None
    lib.ccfr_batch_footprint.restype = i64
    lib.ccfr_batch_footprint.argtypes = [i32, i32, i32]
    lib.ccfr_batch_add.argtypes = [vp, i32, vp, i32, vp, i32, vp, vp, vp, vp, C.POINTER(StepParams),
                                   C.POINTER(i32), vp]
    lib.ccfr_batch_remove.argtypes = [vp, i32, vp]
    lib.ccfr_batch_step.argtypes = [vp, vp]
    lib.ccfr_batch_rollback.argtypes = [vp, vp]
    lib.ccfr_batch_read.argtypes = [vp, i32, vp, vp, vp]
    lib.ccfr_batch_stats.argtypes = [vp, C.POINTER(i32), C.POINTER(i64)]
    _lib = lib
    return lib


def _check(code, where):
    if code != 0:
        raise CcfrError(code, where)


def _dev(t, dtype: str, numel: int, name: str, optional: bool = False):
    """Device pointer of `t` after checking it is a contiguous device tensor of
    `dtype` ("float32", "int32", "uint8") holding exactly `numel` elements: the
    kernels index these buffers by the mesh's sizes, so a shorter buffer would
    be read or written past its end."""
    if t is None:
        if optional or numel == 0:
            return None
        raise ValueError(f"{name}: a device tensor is required")
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{name}: must be a device tensor")
    if str(t.dtype) != "torch." + dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if t.numel() != numel:
        raise ValueError(f"{name}: {t.numel()} elements, expected {numel}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    return C.c_void_p(t.data_ptr()) if numel else None


def _host_exact(a, dtype, rows: int, cols: int, name: str):
    """Host array of exactly rows x cols elements (cols = 1: a vector)."""
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype)
    if a.size != rows * cols:
        raise ValueError(f"{name}: {a.size} elements, expected {rows * cols}")
    return a, a.ctypes.data_as(C.c_void_p)


def _host(a, dtype):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype)
    return a, a.ctypes.data_as(C.c_void_p)


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def make_params(p) -> Params:
    """From anything with r, xi, delta, guard, eps_retract, eps_plesnik, max_passes
    (and optionally response, resp_compliance, vis_width, mu_s, mu_k)."""
    g = lambda name: float(getattr(p, name, 0.0))
    return Params(p.r, p.xi, p.delta, p.guard, p.eps_retract, p.eps_plesnik, int(p.max_passes),
                  FLAG_RESPONSE if getattr(p, "response", False) else 0, g("resp_compliance"), g("vis_width"),
                  g("mu_s"), g("mu_k"))


def make_step_params(step, p) -> StepParams:
    return StepParams(step.dt, (C.c_float * 3)(*step.gravity), int(step.iters), step.alpha, make_params(p),
                      int(bool(getattr(step, "early_exit", False))), float(getattr(step, "conv_tol", 0.0)))


class Context:
    def __init__(self, device: int = 0):
        self.lib = load()
        h = C.c_void_p()
        _check(self.lib.ccfr_create(C.byref(h), int(device)), "ccfr_create")
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            self.lib.ccfr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, vf=0, ee=0, vv=0, contacts=0, halfspaces=0, ve=0, stream=None):
        _check(self.lib.ccfr_reserve(self.h, int(vf), int(ee), int(vv), int(ve), int(contacts), int(halfspaces),
                                     _stream(stream)), "ccfr_reserve")

    def sync_status(self, reset=False, stream=None, raise_on_error=False):
        info = StatusInfo()
        code = self.lib.ccfr_sync_status(self.h, _stream(stream), C.byref(info), int(bool(reset)))
        if code == -3 or (raise_on_error and code != 0):
            raise CcfrError(code, "ccfr_sync_status")
        return code, {
            "status_bits": int(info.status_bits),
            "last_counts": list(info.last_counts),
            "last_contacts": int(info.last_contacts),
            "last_halfspaces": int(info.last_halfspaces),
            "need": list(info.need),
            "totals": list(info.totals),
            "candidate_builds": int(info.candidate_builds),
            "iterations_run": int(info.iterations_run),
            "halt_runs": list(info.halt_runs),
            "max_halt_run": int(info.max_halt_run),
            "last_ve": int(info.last_ve),
            "need_ve": int(info.need_ve),
            "total_ve": int(info.total_ve),
        }


    def grow(self, info, factor=1.5):
        """Reserve the list sizes a CAPACITY status reported (info from sync_status).
        A primitive too large to bin (status bit 16) is not fixed by larger
        lists: that raises CcfrError."""
        if info["status_bits"] & 16:
            raise CcfrError(-2, "a primitive's box is too large to bin (coordinates out of range)")
        nd = info["need"]
        self.reserve(vf=int(nd[0] * factor) + 1024, ee=int(nd[1] * factor) + 1024, vv=int(nd[2] * factor) + 1024,
                     ve=int(info.get("need_ve", 0) * factor) + 1024, contacts=int(nd[3] * factor) + 1024,
                     halfspaces=int(nd[4] * factor) + 1024)

    def set_tuning(self, cell_scale=None, pair_split=None, pair_reuse=None, pair_skin=None, broad_phase=None,
                   direct_regions=None):
        """Change any of the speed-only knobs (None keeps the current value)."""
        cur = self.get_tuning()
        t = Tuning(float(cur["cell_scale"] if cell_scale is None else cell_scale),
                   int(cur["pair_split"] if pair_split is None else pair_split),
                   int(cur["pair_reuse"] if pair_reuse is None else pair_reuse),
                   int(cur["pair_skin"] if pair_skin is None else pair_skin),
                   int(cur["broad_phase"] if broad_phase is None else broad_phase),
                   int(cur["direct_regions"] if direct_regions is None else direct_regions))
        _check(self.lib.ccfr_set_tuning(self.h, C.byref(t)), "ccfr_set_tuning")

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(self.lib.ccfr_get_tuning(self.h, C.byref(t)), "ccfr_get_tuning")
        return {"cell_scale": float(t.cell_scale), "pair_split": int(t.pair_split),
                "pair_reuse": int(t.pair_reuse), "pair_skin": int(t.pair_skin), "broad_phase": int(t.broad_phase),
                "direct_regions": int(t.direct_regions)}

    def profile_enable(self, on=True):
        _check(self.lib.ccfr_profile_enable(self.h, int(bool(on))), "ccfr_profile_enable")

    def profile_read(self, stream=None):
        """(ms per stage [6], launches per stage [6]) of the most recent substep."""
        ms = np.zeros(6, np.float32)
        n = np.zeros(6, np.int32)
        _check(self.lib.ccfr_profile_read(self.h, _stream(stream), ms.ctypes.data_as(C.c_void_p),
                                          n.ctypes.data_as(C.c_void_p)), "ccfr_profile_read")
        return ms, n


STAGES = ["grid_build", "pair_emission", "contacts", "region_fill", "stretch", "projection"]


class Mesh:
    """Device copy of a mesh (topology, inverse masses, stretch data)."""

    def __init__(self, ctx: Context, n_verts, tris, edges, inv_mass, rest_x=None):
        self.ctx = ctx
        lib = ctx.lib
        tris_a, tris_p = _host(np.asarray(tris).reshape(-1, 3), np.int32)
        edges_a, edges_p = _host(None if edges is None else np.asarray(edges).reshape(-1, 2), np.int32)
        w_a, w_p = _host_exact(inv_mass, np.float32, n_verts, 1, "inv_mass")
        r_a, r_p = _host_exact(rest_x, np.float32, n_verts, 3, "rest_x")
        h = C.c_void_p()
        _check(lib.ccfr_mesh_create(ctx.h, int(n_verts), tris_p, len(tris_a), edges_p,
                                    0 if edges_a is None else len(edges_a), w_p, r_p, C.byref(h)),
               "ccfr_mesh_create")
        self.h = h
        self.n_verts = int(n_verts)
        ne = C.c_int32()
        lib.ccfr_mesh_edges(h, C.byref(ne), None)
        self.n_edges = int(ne.value)

    def edges(self) -> np.ndarray:
        out = np.zeros((self.n_edges, 2), np.int32)
        ne = C.c_int32()
        self.ctx.lib.ccfr_mesh_edges(self.h, C.byref(ne), out.ctypes.data_as(C.c_void_p))
        return out

    def close(self):
        if self.h:
            self.ctx.lib.ccfr_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mesh_from_scene(ctx: Context, scene, stretch=True) -> Mesh:
    return Mesh(ctx, scene.n_verts, scene.tris, scene.edges, scene.inv_mass,
                scene.rest_x if stretch else None)


def batch_footprint(n_verts, n_tris, n_edges) -> int:
    """Device bytes a mesh of these sizes adds to a batch (an upper bound)."""
    return int(load().ccfr_batch_footprint(int(n_verts), int(n_tris), int(n_edges)))


class Batch:
    """Many independent meshes stepped by one set of launches (slot ids as mesh ids)."""

    def __init__(self, ctx: Context, max_slots, max_verts, max_tris, max_edges):
        self.ctx = ctx
        h = C.c_void_p()
        _check(ctx.lib.ccfr_batch_create(ctx.h, int(max_slots), int(max_verts), int(max_tris), int(max_edges),
                                         C.byref(h)), "ccfr_batch_create")
        self.h = h
        self.sizes = {}

    def add(self, n_verts, tris, edges, inv_mass, rest_x, x, v, step_params: StepParams, stream=None) -> int:
        """Admit a mesh; returns its slot.  Raises CcfrError (CAPACITY when it does not fit)."""
        tris_a, tris_p = _host(np.asarray(tris).reshape(-1, 3), np.int32)
        edges_a, edges_p = _host(None if edges is None else np.asarray(edges).reshape(-1, 2), np.int32)
        w_a, w_p = _host_exact(inv_mass, np.float32, n_verts, 1, "inv_mass")
        r_a, r_p = _host_exact(rest_x, np.float32, n_verts, 3, "rest_x")
        x_a, x_p = _host_exact(x, np.float32, n_verts, 3, "x")
        v_a, v_p = _host_exact(v, np.float32, n_verts, 3, "v")
        slot = C.c_int32(-1)
        _check(self.ctx.lib.ccfr_batch_add(self.h, int(n_verts), tris_p, len(tris_a), edges_p,
                                           0 if edges_a is None else len(edges_a), w_p, r_p, x_p, v_p,
                                           C.byref(step_params), C.byref(slot), _stream(stream)), "ccfr_batch_add")
        self.sizes[int(slot.value)] = int(n_verts)
        return int(slot.value)

    def add_scene(self, scene, step_params: StepParams, stretch=True, stream=None) -> int:
        return self.add(scene.n_verts, scene.tris, scene.edges, scene.inv_mass,
                        scene.rest_x if stretch else None, scene.x, scene.v, step_params, stream)

    def remove(self, slot, stream=None):
        _check(self.ctx.lib.ccfr_batch_remove(self.h, int(slot), _stream(stream)), "ccfr_batch_remove")
        self.sizes.pop(int(slot), None)

    def step(self, stream=None):
        _check(self.ctx.lib.ccfr_batch_step(self.h, _stream(stream)), "ccfr_batch_step")

    def rollback(self, stream=None):
        _check(self.ctx.lib.ccfr_batch_rollback(self.h, _stream(stream)), "ccfr_batch_rollback")

    def read(self, slot, stream=None):
        n = self.sizes[int(slot)]
        x = np.zeros((n, 3), np.float32)
        v = np.zeros((n, 3), np.float32)
        _check(self.ctx.lib.ccfr_batch_read(self.h, int(slot), x.ctypes.data_as(C.c_void_p),
                                            v.ctypes.data_as(C.c_void_p), _stream(stream)), "ccfr_batch_read")
        return x, v

    def stats(self):
        n = C.c_int32()
        nv = C.c_int64()
        _check(self.ctx.lib.ccfr_batch_stats(self.h, C.byref(n), C.byref(nv)), "ccfr_batch_stats")
        return int(n.value), int(nv.value)

    def close(self):
        if self.h:
            self.ctx.lib.ccfr_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_candidates(ctx: Context, mesh: Mesh, x, params, stream=None) -> Candidates:
    out = Candidates()
    prm = params if isinstance(params, Params) else make_params(params)
    xp = _dev(x, "float32", 3 * mesh.n_verts, "x")
    _check(ctx.lib.ccfr_build_candidates(ctx.h, mesh.h, xp, C.byref(prm), C.byref(out), _stream(stream)),
           "ccfr_build_candidates")
    return out


def build_regions(ctx: Context, mesh: Mesh, x, cands: Candidates, params, stream=None) -> Regions:
    out = Regions()
    prm = params if isinstance(params, Params) else make_params(params)
    xp = _dev(x, "float32", 3 * mesh.n_verts, "x")
    _check(ctx.lib.ccfr_build_regions(ctx.h, mesh.h, xp, C.byref(cands), C.byref(prm), C.byref(out),
                                      _stream(stream)), "ccfr_build_regions")
    return out


def project_displacements(ctx: Context, regions: Regions, inv_mass, y_in, params, y_out, halted=None,
                          stream=None):
    prm = params if isinstance(params, Params) else make_params(params)
    n = int(regions.n_verts)
    wp = _dev(inv_mass, "float32", n, "inv_mass")
    yp = _dev(y_in, "float32", 3 * n, "y_in")
    op = _dev(y_out, "float32", 3 * n, "y_out")
    hp = _dev(halted, "uint8", n, "halted", optional=True)
    _check(ctx.lib.ccfr_project_displacements(ctx.h, C.byref(regions), wp, yp, C.byref(prm), op, hp,
                                              _stream(stream)),
           "ccfr_project_displacements")


def apply_response(ctx: Context, regions: Regions, inv_mass, y_in, params, dt, y_out, stream=None):
    """applyResponse of Alg. 4 (soft response, visibility weights, friction) on
    the regions; y_out may be y_in."""
    prm = params if isinstance(params, Params) else make_params(params)
    n = int(regions.n_verts)
    wp = _dev(inv_mass, "float32", n, "inv_mass")
    yp = _dev(y_in, "float32", 3 * n, "y_in")
    op = _dev(y_out, "float32", 3 * n, "y_out")
    _check(ctx.lib.ccfr_apply_response(ctx.h, C.byref(regions), wp, yp, C.byref(prm), float(dt), op,
                                       _stream(stream)),
           "ccfr_apply_response")


def project_displacements_noalloc(regions: Regions, inv_mass, y_in, params, y_out, halted=None, status=None,
                                  stream=None):
    """ccfr_project_displacements_noalloc: the projection without a context and
    without any allocation (status: optional device uint32 of one element)."""
    lib = load()
    prm = params if isinstance(params, Params) else make_params(params)
    n = regions.n_verts
    wp = _dev(inv_mass, "float32", n, "inv_mass")
    yp = _dev(y_in, "float32", 3 * n, "y_in")
    op = _dev(y_out, "float32", 3 * n, "y_out")
    hp = _dev(halted, "uint8", n, "halted", optional=True)
    sp = _dev(status, "int32", 1, "status", optional=True)
    _check(lib.ccfr_project_displacements_noalloc(C.byref(regions), wp, yp, C.byref(prm), op, hp, sp,
                                                  _stream(stream)),
           "ccfr_project_displacements_noalloc")


def xpbd_step(ctx: Context, mesh: Mesh, x, v, step_params: StepParams, stream=None):
    xp = _dev(x, "float32", 3 * mesh.n_verts, "x")
    vp = _dev(v, "float32", 3 * mesh.n_verts, "v")
    _check(ctx.lib.ccfr_xpbd_step(ctx.h, mesh.h, xp, vp, C.byref(step_params), _stream(stream)),
           "ccfr_xpbd_step")


def xpbd_step_traced(ctx: Context, mesh: Mesh, x, v, step_params: StepParams, trace, stream=None):
    """xpbd_step that writes the anchor after every iteration into `trace`
    ([iters][n_verts][3] float32 on the device)."""
    xp = _dev(x, "float32", 3 * mesh.n_verts, "x")
    vp = _dev(v, "float32", 3 * mesh.n_verts, "v")
    tp = _dev(trace, "float32", 3 * mesh.n_verts * max(step_params.iters, 1), "trace")
    _check(ctx.lib.ccfr_xpbd_step_traced(ctx.h, mesh.h, xp, vp, C.byref(step_params), tp, _stream(stream)),
           "ccfr_xpbd_step_traced")


def caller_candidates(vf, ee, vv, counts, ve=None) -> Candidates:
    """Candidates view over caller-owned device tensors ([P][2] int32 each, counts [4] int32:
    |VF|, |EE|, |VV|, |VE|; ve None: no particle-edge pairs, counts[3] must be 0).
    The view keeps the tensors alive."""
    lists = (("vf", vf), ("ee", ee), ("vv", vv)) + ((("ve", ve),) if ve is not None else ())
    for name, t in lists:
        _dev(t, "int32", t.numel(), name)
        if t.dim() != 2 or t.shape[1] != 2:
            raise ValueError(f"{name}: shape {tuple(t.shape)}, expected [P][2]")
    _dev(counts, "int32", 4, "counts")
    c = Candidates(vf.data_ptr(), ee.data_ptr(), vv.data_ptr(), counts.data_ptr(), vf.shape[0], ee.shape[0],
                   vv.shape[0], ve.data_ptr() if ve is not None else None, ve.shape[0] if ve is not None else 0)
    c._keep = (vf, ee, vv, counts, ve)
    return c


def caller_regions(offsets, hs_bytes) -> Regions:
    """Regions view over caller-owned device tensors: offsets [N+1] int32, hs_bytes [H*32] uint8.
    The view keeps the tensors alive."""
    if offsets.dim() != 1 or offsets.shape[0] < 1:
        raise ValueError("offsets: expected [N+1]")
    _dev(offsets, "int32", offsets.numel(), "offsets")
    _dev(hs_bytes, "uint8", hs_bytes.numel(), "hs_bytes")
    if hs_bytes.numel() % 32:
        raise ValueError("hs_bytes: not a whole number of 32-byte half-spaces")
    r = Regions(offsets.shape[0] - 1, 0, offsets.data_ptr(), hs_bytes.data_ptr(), hs_bytes.numel() // 32)
    r._keep = (offsets, hs_bytes)
    return r


# ---- copying device lists back (for tests and counters) ----

def _dev_view(ptr, count, dtype, device):
    """Copy `count` elements of dtype from a device pointer into a host numpy array."""
    import torch
    nbytes = int(count) * np.dtype(dtype).itemsize
    if nbytes == 0:
        return np.zeros(0, dtype)
    host = torch.empty(nbytes, dtype=torch.uint8)
    dst = host.data_ptr()
    # device-to-host copy through the HIP runtime torch already loaded
    hip = _hiprt()
    rc = hip.hipMemcpy(C.c_void_p(dst), C.c_void_p(ptr), C.c_size_t(nbytes), 2)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed: {rc}")
    return host.numpy().view(dtype).copy()


_hip = None


def _hiprt():
    global _hip
    if _hip is None:
        for name in ("libamdhip64.so", "libamdhip64.so.7", "libamdhip64.so.6"):
            try:
                _hip = C.CDLL(name)
                break
            except OSError:
                continue
        if _hip is None:
            raise RuntimeError("libamdhip64 not found")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    return _hip


def read_candidates(c: Candidates) -> dict:
    """Synchronous copy of the candidate lists (the stream must be synchronised)."""
    counts = _dev_view(c.counts_dev, 4, np.int32, None)
    caps = (c.cap_vf, c.cap_ee, c.cap_vv, c.cap_ve)
    out = {}
    for k, (name, ptr) in enumerate((("vf", c.vf), ("ee", c.ee), ("vv", c.vv), ("ve", c.ve))):
        n = int(counts[k])
        if n > caps[k]:
            raise CcfrError(-2, f"{name} list overflow ({n} > {caps[k]})")
        out[name] = _dev_view(ptr, 2 * n, np.int32, None).reshape(-1, 2)
    out["counts"] = counts
    return out


def read_regions(r: Regions):
    """Synchronous copy: (offsets [N+1] int32, half-spaces [H] HALFSPACE_DTYPE)."""
    off = _dev_view(r.offsets, r.n_verts + 1, np.int32, None)
    H = int(off[-1])
    if H > r.cap:
        raise CcfrError(-2, f"half-space overflow ({H} > {r.cap})")
    hs = _dev_view(r.hs, H * 32, np.uint8, None).view(HALFSPACE_DTYPE)
    return off, hs
