"""Autotuner of the speed-only knobs of a context.

The knobs are the grid cell size (`cell_scale`, a multiple of the default
cell: 1.2 x the typical edge length + 2 pad), the number of lanes that share
one broad-phase query (`pair_split`) and how solver iterations share candidate
builds inside a substep: a fixed number per build (`pair_reuse`) or as many as
the measured motion allows within a widening of s r (`pair_skin` = s), and
the broad phase itself (`broad_phase`: the hash grid, or the bounding-volume
hierarchy, which has no cell or split knob), and whether the narrow phase
writes a substep's slot regions itself (`direct_regions`, tried on the best
of the other settings).  Smaller cells put
fewer entries in the buckets a query scans but bin long primitives one level
up; more lanes per query shorten the walks of queries in dense folds at the
price of more lanes; sharing a build saves grid builds and queries at the price
of longer lists (the boxes are widened by the motion the shared iterations can
make).  The best values depend on the mesh's edge lengths, its contact density
and the pad.  Every setting gives the same regions and results, so the tuner
only times: it runs the same work once per setting, keeps the fastest, and
caches the choice per size class in a JSON file.
"""
from __future__ import annotations

import json
import math
import os
import sys

from . import ccfr

CELL_SCALES = (0.35, 0.5, 0.6, 0.7, 0.85, 1.0, 1.2)
PAIR_SPLITS = (1, 3, 9)
# (pair_reuse, pair_skin): fixed groups of 1-4 iterations, or builds that follow
# the motion with a skin of 1-3 r
PAIR_MODES = ((1, 0), (2, 0), (3, 0), (4, 0), (1, 1), (1, 2), (1, 3))
BROAD_PHASES = (0, 1)
DIRECT_REGIONS = (0, 1)


def size_class(n_verts, n_tris, n_edges, r, kind="mesh") -> str:
    """Key of a workload shape: log2 sizes and the pad's order of magnitude."""
    def lg(v):
        return int(math.ceil(math.log2(max(int(v), 1))))
    return f"{kind}-v{lg(n_verts)}-t{lg(n_tris + 1)}-e{lg(n_edges + 1)}-r{int(round(math.log10(max(r, 1e-9))))}"


def default_cache_path() -> str:
    return os.environ.get("CCFR_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "ccfr", "tuning.json"))


class Cache:
    def __init__(self, path: str | None = None):
        self.path = path or default_cache_path()
        self.data = {}
        if os.path.exists(self.path):
            try:
                with open(self.path) as f:
                    self.data = json.load(f)
            except (OSError, ValueError):
                self.data = {}

    def get(self, key):
        return self.data.get(key)

    def put(self, key, value):
        self.data[key] = value
        try:
            os.makedirs(os.path.dirname(self.path), exist_ok=True)
            with open(self.path, "w") as f:
                json.dump(self.data, f, indent=1, sort_keys=True)
        except OSError:
            pass


class TooLarge(Exception):
    """A setting whose lists would outgrow the tuner's memory limit."""


def list_bytes(info) -> int:
    """Device bytes of the lists a status record's needs call for."""
    nd = info["need"]
    return 8 * (nd[0] + nd[1] + nd[2]) + 32 * nd[3] + 44 * nd[4]


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _settings(candidates, splits, modes, broad_phases):
    """(cell scale, split, reuse, skin, broad phase) to time: the grid at every
    cell scale and split, the hierarchy (no cell or split knob) once per mode."""
    for bp in broad_phases:
        for c in (candidates if bp == 0 else (1.0,)):
            for sp in (splits if bp == 0 else (1,)):
                for ru, sk in modes:
                    yield c, sp, ru, sk, bp


def tune(ctx: ccfr.Context, run, candidates=CELL_SCALES, splits=PAIR_SPLITS, modes=((1, 0),),
         repeats: int = 2, log=_log, grow_factor: float = 4.0, broad_phases=(0,), directs=(0,)) -> dict:
    """Time `run(limit)` (device milliseconds of a fixed piece of work, starting
    from the same state every call, and the list bytes it needed) under each
    (cell scale, split, (reuse, skin), broad phase); leave the fastest set.  A
    setting whose lists would need more than grow_factor times those of the
    first setting is skipped (run raises TooLarge), and one whose first timing
    is three times the best so far is not timed again."""
    times = {}
    limit = None
    best_ms = math.inf
    for key in _settings(candidates, splits, modes, broad_phases):
        c, sp, ru, sk, bp = key
        ctx.set_tuning(cell_scale=c, pair_split=sp, pair_reuse=ru, pair_skin=sk, broad_phase=bp)
        try:
            ms, nbytes = run(limit)     # records the graph for this setting
            if limit is None:
                limit = grow_factor * max(nbytes, 1 << 28)
            if ms < 3.0 * best_ms:
                ms = min(run(limit)[0] for _ in range(repeats))
        except TooLarge:
            ms = math.inf
        times[key] = ms
        best_ms = min(best_ms, ms)
        if log:
            log(f"[tune] cell {c} split {sp} reuse {ru} skin {sk} broad phase {bp}: {ms:.3f} ms")
    best = min(times, key=times.get)
    times = {k + (directs[0],): v for k, v in times.items()}
    best = best + (directs[0],)
    for d in directs[1:]:
        key = best[:5] + (d,)
        ctx.set_tuning(cell_scale=key[0], pair_split=key[1], pair_reuse=key[2], pair_skin=key[3], broad_phase=key[4],
                       direct_regions=d)
        try:
            run(limit)
            ms = min(run(limit)[0] for _ in range(repeats))
        except TooLarge:
            ms = math.inf
        times[key] = ms
        if log:
            log(f"[tune] best setting with direct regions {d}: {ms:.3f} ms")
        if ms < times[best]:
            best = key
    ctx.set_tuning(cell_scale=best[0], pair_split=best[1], pair_reuse=best[2], pair_skin=best[3],
                   broad_phase=best[4], direct_regions=best[5])
    return {"cell_scale": best[0], "pair_split": best[1], "pair_reuse": best[2], "pair_skin": best[3],
            "broad_phase": best[4], "direct_regions": best[5],
            "ms": {"/".join(str(q) for q in k): v for k, v in times.items()}}


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def tune_mesh(ctx: ccfr.Context, mesh: ccfr.Mesh, x, v, sp: ccfr.StepParams, steps: int = 4,
              candidates=CELL_SCALES, splits=PAIR_SPLITS, modes=PAIR_MODES, cache: Cache | None = None,
              key: str | None = None, log=_log, broad_phases=BROAD_PHASES, directs=DIRECT_REGIONS) -> dict:
    """Tune on `steps` single-mesh steps from the state (x, v), which is restored."""
    import torch
    if cache is not None and key is not None:
        hit = cache.get(key)
        if hit is not None:
            ctx.set_tuning(cell_scale=hit["cell_scale"], pair_split=hit["pair_split"],
                           pair_reuse=hit.get("pair_reuse", 1), pair_skin=hit.get("pair_skin", 0),
                           broad_phase=hit.get("broad_phase", 0), direct_regions=hit.get("direct_regions", 0))
            return dict(hit, cached=True)
    x0, v0 = x.clone(), v.clone()

    def run(limit=None):
        for _ in range(4):
            x.copy_(x0)
            v.copy_(v0)
            e0, e1 = _events()
            e0.record()
            for _ in range(steps):
                ccfr.xpbd_step(ctx, mesh, x, v, sp)
            e1.record()
            code, info = ctx.sync_status(reset=True)
            if code == 0:
                return e0.elapsed_time(e1), list_bytes(info)
            if code != -2:
                raise ccfr.CcfrError(code, "tuning run")
            if limit is not None and list_bytes(info) > limit:
                raise TooLarge()
            ctx.grow(info)                      # lists too small: grow and time again
        raise ccfr.CcfrError(-2, "tuning run")

    out = tune(ctx, run, candidates, splits, modes, log=log, broad_phases=broad_phases, directs=directs)
    x.copy_(x0)
    v.copy_(v0)
    torch.cuda.synchronize()
    if cache is not None and key is not None:
        cache.put(key, out)
    return dict(out, cached=False)


def tune_batch(ctx: ccfr.Context, batch: ccfr.Batch, candidates=CELL_SCALES, splits=PAIR_SPLITS,
               modes=PAIR_MODES, log=_log, directs=(0,)) -> dict:
    """Tune on one step of the resident batch; every trial is rolled back."""
    def run(limit=None):
        for _ in range(4):
            e0, e1 = _events()
            e0.record()
            batch.step()
            e1.record()
            code, info = ctx.sync_status(reset=True)
            batch.rollback()
            if code == 0:
                return e0.elapsed_time(e1), list_bytes(info)
            if code != -2:
                raise ccfr.CcfrError(code, "tuning run")
            if limit is not None and list_bytes(info) > limit:
                raise TooLarge()
            ctx.grow(info)
        raise ccfr.CcfrError(-2, "tuning run")

    return tune(ctx, run, candidates, splits, modes, log=log, directs=directs)
