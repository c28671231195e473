"""Continuous-batching request loop over the batched substep.

Simulation requests (a mesh, its initial state, its step parameters and a
number of steps) arrive over time.  The loop keeps every admitted request's
positions, velocities and topology resident in one device batch and steps all
of them with one recorded graph per step.  Between steps it retires the
requests that have run all their steps and admits waiting ones, first come
first served, while the sum of their device footprints stays within a byte
budget and the batch has a free slot and pool space.  A request that arrives
while others run joins at the next step boundary, so its steps overlap theirs
on the device.

The batch shares its context's workspace; when a workspace list overflows
(the device reports CAPACITY), the loop grows the list to the reported need,
restores the step's entry state and runs the step again, so no step is ever
kept with dropped contacts.

`run_sequential` is the one-mesh-at-a-time alternative: each request, in
arrival order, runs alone through the single-mesh step.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import ccfr


@dataclass
class Job:
    """One request: `scene` carries mesh, state, collision and step parameters."""
    id: int
    arrival: float          # seconds after the start of the run
    scene: object
    steps: int


@dataclass
class JobResult:
    id: int
    n_verts: int
    n_dynamic: int
    steps: int
    arrival: float
    admitted: float = 0.0
    finished: float = 0.0
    x: np.ndarray | None = None
    v: np.ndarray | None = None


@dataclass
class RunStats:
    mode: str
    makespan_s: float = 0.0
    busy_s: float = 0.0
    updates: int = 0
    step_ms: list = field(default_factory=list)          # one entry per launched step
    request_step_ms: list = field(default_factory=list)  # one entry per (request, step)
    request_latency_s: list = field(default_factory=list)
    max_resident: int = 0
    max_resident_verts: int = 0
    retries: int = 0
    tuning: dict | None = None
    results: dict = field(default_factory=dict)

    def summary(self) -> dict:
        def pct(a, q):
            return float(np.percentile(np.asarray(a), q)) if len(a) else 0.0
        return {
            "mode": self.mode,
            "requests": len(self.results),
            "makespan_s": self.makespan_s,
            "gpu_busy_s": self.busy_s,
            "vertex_updates": self.updates,
            "throughput": self.updates / self.makespan_s if self.makespan_s > 0 else 0.0,
            "busy_throughput": self.updates / self.busy_s if self.busy_s > 0 else 0.0,
            "launched_steps": len(self.step_ms),
            "p50_step_ms": pct(self.step_ms, 50),
            "p99_step_ms": pct(self.step_ms, 99),
            "p50_request_step_ms": pct(self.request_step_ms, 50),
            "p99_request_step_ms": pct(self.request_step_ms, 99),
            "p50_request_latency_s": pct(self.request_latency_s, 50),
            "p99_request_latency_s": pct(self.request_latency_s, 99),
            "max_resident_requests": self.max_resident,
            "max_resident_verts": self.max_resident_verts,
            "capacity_retries": self.retries,
            "tuning": self.tuning,
        }


def footprint(scene) -> int:
    return ccfr.batch_footprint(scene.n_verts, len(scene.tris), len(scene.edges))


def _grow(ctx, info):
    ctx.grow(info)


class _GpuTimer:
    """Device time of the work enqueued between start() and stop() on the current stream."""

    def __init__(self):
        import torch
        self.torch = torch
        self.stream = torch.cuda.current_stream()

    def start(self):
        self.e0 = self.torch.cuda.Event(enable_timing=True)
        self.e1 = self.torch.cuda.Event(enable_timing=True)
        self.e0.record(self.stream)

    def stop(self):
        self.e1.record(self.stream)

    def ms(self):
        return self.e0.elapsed_time(self.e1)


class _HostTimer:
    def start(self):
        self.t0 = time.perf_counter()

    def stop(self):
        self.t1 = time.perf_counter()

    def ms(self):
        return 1e3 * (self.t1 - self.t0)


class Server:
    """Continuous batching within `budget_bytes` of per-request device footprint.

    `batch` (default: a new ccfr.Batch sized from the budget) needs add_scene,
    step, rollback, read and remove; `timer` (default: HIP events) times each
    launched step."""

    def __init__(self, ctx, budget_bytes: int, max_slots: int = 4096, max_verts: int | None = None,
                 max_tris: int | None = None, max_edges: int | None = None, batch=None, timer=None,
                 footprint_fn=None, tune_at: int | None = None, step_verts_cap: int | None = None):
        """tune_at: once this many requests are resident, pick the grid cell
        size by timing one rolled-back step per candidate (autotune).
        step_verts_cap: no request is admitted while the resident vertices
        would exceed this many (a step's time, which every resident request
        waits for, grows with them); a request larger than the cap runs alone."""
        self.ctx = ctx
        self.tune_at = tune_at
        self.step_verts_cap = step_verts_cap
        self.tuning = None
        self.budget = int(budget_bytes)
        self.footprint = footprint_fn or footprint
        if batch is None:
            # pool sizes: what the budget can hold at the smallest per-vertex footprint
            per_v = max(footprint_per_vertex(), 1)
            nv = max_verts if max_verts is not None else max(self.budget // per_v, 4096)
            batch = ccfr.Batch(ctx, max_slots, nv, max_tris if max_tris is not None else 2 * nv,
                               max_edges if max_edges is not None else 3 * nv)
        self.batch = batch
        self.timer = timer or _GpuTimer()

    def close(self):
        self.batch.close()

    def run(self, jobs: list[Job], keep_results: bool = False, clock=time.perf_counter,
            sleep=time.sleep) -> RunStats:
        st = RunStats("batched")
        jobs = sorted(jobs, key=lambda j: (j.arrival, j.id))
        waiting: list[Job] = []
        resident: dict[int, tuple[Job, int, int, JobResult]] = {}   # slot -> (job, steps done, fp, result)
        used = 0
        nxt = 0
        t0 = clock()
        while nxt < len(jobs) or waiting or resident:
            now = clock() - t0
            tw0 = clock()
            while nxt < len(jobs) and jobs[nxt].arrival <= now:
                waiting.append(jobs[nxt])
                nxt += 1
            # admission, first come first served
            resident_verts = sum(r[0].scene.n_verts for r in resident.values())
            while waiting:
                j = waiting[0]
                fp = self.footprint(j.scene)
                if used + fp > self.budget and resident:
                    break
                if (self.step_verts_cap is not None and resident
                        and resident_verts + j.scene.n_verts > self.step_verts_cap):
                    break
                sp = ccfr.make_step_params(j.scene.step, j.scene.params)
                try:
                    slot = self.batch.add_scene(j.scene, sp)
                except ccfr.CcfrError as e:
                    if e.code == -2 and resident:          # no slot or pool space now
                        break
                    raise
                waiting.pop(0)
                used += fp
                resident_verts += j.scene.n_verts
                res = JobResult(j.id, j.scene.n_verts, j.scene.n_dynamic, j.steps, j.arrival,
                                admitted=clock() - t0)
                resident[slot] = (j, 0, fp, res)
            if not resident:
                if nxt < len(jobs):
                    sleep(max(0.0, jobs[nxt].arrival - (clock() - t0)))
                continue
            st.max_resident = max(st.max_resident, len(resident))
            if self.tune_at is not None and self.tuning is None and len(resident) >= self.tune_at:
                from . import autotune
                # a short search: every setting re-records the step graph while requests wait
                self.tuning = autotune.tune_batch(self.ctx, self.batch, candidates=(0.7, 0.85, 1.0), splits=(1,),
                                                  modes=((1, 0), (2, 0)), directs=(0, 1))
            st.max_resident_verts = max(st.max_resident_verts, sum(r[0].scene.n_verts for r in resident.values()))
            # one step of every resident request
            while True:
                self.timer.start()
                self.batch.step()
                self.timer.stop()
                code, info = self.ctx.sync_status(reset=True)
                if code == 0:
                    break
                if code != -2:
                    raise ccfr.CcfrError(code, "batched step")
                _grow(self.ctx, info)
                self.batch.rollback()
                st.retries += 1
            ms = self.timer.ms()
            st.step_ms.append(ms)
            st.busy_s += ms * 1e-3
            tnow = clock() - t0
            # what a resident request waits for one of its steps: admission
            # work of this round, the step itself and the status read
            wall_ms = 1e3 * (clock() - tw0)
            for slot in list(resident):
                j, done, fp, res = resident[slot]
                done += 1
                st.request_step_ms.append(wall_ms)
                st.updates += j.scene.n_dynamic * j.scene.step.iters
                if done >= j.steps:
                    if keep_results:
                        res.x, res.v = self.batch.read(slot)
                    self.batch.remove(slot)
                    res.finished = tnow
                    st.request_latency_s.append(tnow - j.arrival)
                    st.results[j.id] = res
                    used -= fp
                    del resident[slot]
                else:
                    resident[slot] = (j, done, fp, res)
        st.makespan_s = clock() - t0
        st.tuning = self.tuning
        return st


def footprint_per_vertex() -> int:
    """Smallest per-vertex footprint among cloth-like meshes (about 2 triangles
    and 3 edges per vertex), used to size the pool from a byte budget."""
    n = 1 << 16
    return ccfr.batch_footprint(n, 2 * n, 3 * n) // n


def run_sequential(ctx: ccfr.Context, jobs: list[Job], keep_results: bool = False,
                   clock=time.perf_counter) -> RunStats:
    """Each request alone through the single-mesh step, in arrival order."""
    import torch
    st = RunStats("sequential")
    jobs = sorted(jobs, key=lambda j: (j.arrival, j.id))
    stream = torch.cuda.current_stream()
    t0 = clock()
    for j in jobs:
        now = clock() - t0
        if j.arrival > now:
            time.sleep(j.arrival - now)
        sc = j.scene
        res = JobResult(j.id, sc.n_verts, sc.n_dynamic, j.steps, j.arrival, admitted=clock() - t0)
        mesh = ccfr.mesh_from_scene(ctx, sc)
        x = torch.from_numpy(np.ascontiguousarray(sc.x, np.float32)).cuda()
        v = torch.from_numpy(np.ascontiguousarray(sc.v, np.float32)).cuda()
        sp = ccfr.make_step_params(sc.step, sc.params)
        st.max_resident = 1
        st.max_resident_verts = max(st.max_resident_verts, sc.n_verts)
        x0, v0 = x.clone(), v.clone()
        while True:
            # all steps of the request back to back; status read once at the end
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(j.steps + 1)]
            ev[0].record(stream)
            for k in range(j.steps):
                ccfr.xpbd_step(ctx, mesh, x, v, sp)
                ev[k + 1].record(stream)
            code, info = ctx.sync_status(reset=True)
            if code == 0:
                break
            if code != -2:
                raise ccfr.CcfrError(code, "single-mesh step")
            _grow(ctx, info)
            x.copy_(x0)
            v.copy_(v0)
            st.retries += 1
        for k in range(j.steps):
            ms = ev[k].elapsed_time(ev[k + 1])
            st.step_ms.append(ms)
            st.request_step_ms.append(ms)
            st.busy_s += ms * 1e-3
        st.updates += sc.n_dynamic * sc.step.iters * j.steps
        res.finished = clock() - t0
        st.request_latency_s.append(res.finished - j.arrival)
        if keep_results:
            res.x, res.v = x.cpu().numpy(), v.cpu().numpy()
        st.results[j.id] = res
        mesh.close()
    st.makespan_s = clock() - t0
    return st
