#!/usr/bin/env python3
"""Benchmark of the CCFR hot path on one MI355X.

A step is one XPBD substep of the whole path (Alg. 4): prediction, then per
solver iteration the broad phase (ccfr_build_candidates), the narrow phase
(ccfr_build_regions), one stretch pass and the projection
(ccfr_project_displacements), then the velocity update, all recorded in one HIP
graph.  The default workload is the 65,536-vertex cloth (256 x 256, 2 m) dropped
from 0.1 m onto a static 4 m ground quad with N(0, 0.5 m/s) random initial
velocities, 20 iterations per step, dt = 1/120 s, r = xi = 1 mm; the timed
region is its 60 steps from the initial state.

value = dynamic vertices x solver iterations run / wall time of the timed
region (each update is one vertex through candidates, regions and projection in
one iteration; the stretch pass and the glue kernels are inside the timed
time).  stage_rooflines gives every stage of the path (candidates, regions,
projection) against the HBM peak, from HIP events on the stream in a second
pass over the same steps run as individual launches (events cannot be read back
from inside a replayed graph), with HBM traffic from the committed rocprofv3
summary; roofline repeats the stage with the most time.  cpu_baseline times the
FP64 oracle on a bounded sample of the same workload.  The default line also
carries the coupled codimensional workload (coupled_c5) and the served request
stream against one mesh at a time (served_c4).  Other workloads: --workload c0,
c2, c3, c5, c4 (the served stream as the whole line), c1r (c1 with the soft
response and friction), c2e (c2 with the convergence check).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from paper_2607_26901_amd.scenes import BENCH_KNOBS as S_BENCH_KNOBS

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "vertex region build+project updates/s (65k cloth); p50/p99 step latency"
# the served stream's cap on resident vertices per batched step (a step's time,
# which every resident request waits for, grows with them)
SERVED_VERTS_CAP = 250000
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    from paper_2607_26901_amd import scenes as S
    if name == "c1":
        sc = S.c1()
        desc = ("c1: 256x256-vertex cloth (65,536 dynamic vertices, 130,050 triangles, side 2 m) dropped from "
                "0.1 m onto a static 4 m ground quad, initial velocities N(0, 0.5 m/s), 20 iterations/step, "
                "dt 1/120 s, r = xi = 1 mm, FP32")
    elif name == "c0":
        sc = S.c0()
        desc = "c0: 32x32 cloth (1 m) onto a static 642-vertex icosphere, 10 iterations/step, dt 1/60 s, r = xi = 2 mm"
    elif name == "c3":
        sc = S.c3()
        desc = "c3: 2,000,000 particles in a 1x1x2 m column inside a 12-triangle box, 10 iterations/step"
    elif name == "c2":
        sc = S.c2()
        desc = "c2: 10,000 pinned helical strands x 64 segments (650,000 vertices), edge-edge only"
    elif name == "c1r":
        from dataclasses import replace
        sc = S.c1()
        sc = replace(sc, params=replace(sc.params, delta=5e-4, response=True, resp_compliance=1e-6, vis_width=1e-4,
                                        mu_s=0.4, mu_k=0.3))
        desc = ("c1r: the c1 cloth with the soft response, visibility weights and friction of Sec. 3.3 before every "
                "projection: delta = 0.5 mm (boxes padded by delta / 2 more), compliance 1e-6, visibility width "
                "0.1 mm, mu_s = 0.4, mu_k = 0.3")
    elif name == "c2e":
        from dataclasses import replace
        sc = S.c2()
        sc = replace(sc, step=replace(sc.step, early_exit=True, conv_tol=1e-6))
        desc = ("c2e: the c2 strands with the convergence check of Alg. 4: a substep's iterations end after the "
                "first one in which no vertex falls short of its proposal by more than 1 um (at most 10)")
    elif name == "c5":
        sc = S.c5()
        desc = ("c5: coupled codimensional scene (13,612 vertices): floor, pinned two-layer rod lattice (32 rods x "
                "60 segments over 95 units), two soft tentacled bodies (642-vertex spheres of radius 9, 8 arms of 12 "
                "segments), a 64x64 paper sheet and a 39x39x4 block of free particles, 10 iterations/step, dt 1/120 "
                "s, r = 0.4, xi = 0.06, delta = 0.01 (scene units), all four pair kinds")
    else:
        raise SystemExit(f"unknown workload {name}")
    return sc, desc


# Algorithmic bytes of one solver iteration of each stage of the path: every
# input of the stage read once and every output written once (N vertices, T
# triangles, E edges, P candidate pairs of the method's own box test, H
# half-spaces).  Positions 12 B, inverse masses 4 B, triangles 12 B, edges 8 B,
# a pair 8 B, a half-space 28 B written (n, d, phi, key) and 24 B read
# (n, d, key); the three sum to 60N + 24T + 16E + 16P + 52H.
def stage_bytes(stage, N, T, E, P, H):
    if stage == "a1_candidates":
        # positions and topology in, pairs out
        return 12 * N + 12 * T + 8 * E + 8 * P
    if stage == "a2_regions":
        # pairs, positions, inverse masses and topology in; per-vertex offsets
        # and half-spaces out
        return 8 * P + 12 * N + 4 * N + 12 * T + 8 * E + 4 * N + 28 * H
    if stage == "a4_projection":
        # proposals and inverse masses in, half-spaces read, displacements out
        return 12 * N + 4 * N + 24 * H + 12 * N
    raise KeyError(stage)


# The profiled stages (ccfr.STAGES) that make up each stage of the path.
STAGE_PARTS = {"a1_candidates": ("grid_build", "pair_emission"),
               "a2_regions": ("contacts", "region_fill"),
               "a4_projection": ("projection",)}
# The kernels of each stage, for the counter summary.
STAGE_KERNELS = {"a1_candidates": ("k_reset_build", "k_grid_count", "k_scan_reduce", "k_scan_down",
                                   "k_grid_scatter", "k_pairs"),
                 "a2_regions": ("k_contacts", "k_fill_slots"),
                 "a4_projection": ("k_project_fast", "k_project_slow")}


# Speed knobs the autotuner chose per workload (bench.py --tune, on four steps
# from the middle of the run); the default run times these.  The variants of a
# workload with a row after the core path switched on take its knobs.
TUNED = dict(S_BENCH_KNOBS, c1r=S_BENCH_KNOBS["c1"], c2e=S_BENCH_KNOBS["c2"])


# rocprofv3 summaries of every kernel of a workload (per-dispatch durations,
# copy-scaled FETCH_SIZE / WRITE_SIZE, occupancy), written by
# paper_2607_26901_amd/profiling.py.
KERNEL_PROFILES = {"c1": "profiles/c1_kernels.md"}


def stage_traffic(workload, knobs, stage, dispatches_per_iter):
    """HBM bytes per iteration of a stage's kernels, from the committed counter
    summary (copy-scaled FETCH_SIZE + WRITE_SIZE per dispatch times dispatches
    per iteration), or None if there is no summary, a kernel's source changed
    since it was taken, or it was taken with other knobs."""
    from paper_2607_26901_amd import profiling
    path = KERNEL_PROFILES.get(workload)
    if path is None or not os.path.exists(os.path.join(ROOT, path)):
        return None
    summ = profiling.read_kernel_summary(os.path.join(ROOT, path))
    if not summ or summ.get("knobs") != profiling.knobs_key(knobs):
        return None
    for src, sha in summ.get("sources", {}).items():
        if profiling.sha256(os.path.join(ROOT, src)) != sha:
            return None
    total = 0.0
    for k in STAGE_KERNELS[stage]:
        rec = summ["kernels"].get(k)
        if rec is None or rec.get("traffic_bytes") is None:
            if dispatches_per_iter.get(k, 0) > 0:
                return None
            continue
        total += rec["traffic_bytes"] * dispatches_per_iter.get(k, 0.0)
    return total


def profiled_dispatches(workload, knobs):
    """Dispatches of every kernel per solver iteration in the committed
    profile of the workload (None if there is none for these knobs)."""
    from paper_2607_26901_amd import profiling
    path = KERNEL_PROFILES.get(workload)
    if path is None or not os.path.exists(os.path.join(ROOT, path)):
        return None
    summ = profiling.read_kernel_summary(os.path.join(ROOT, path))
    if not summ or summ.get("knobs") != profiling.knobs_key(knobs) or not summ.get("iterations"):
        return None
    return {k: rec["calls"] / summ["iterations"] for k, rec in summ["kernels"].items()}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sc, budget_s=25.0):
    """The oracle as it stands, one solver iteration of the whole path on the full
    mesh in a folded (contact-rich) state of the same workload, on all host
    threads; and one iteration of the 32x32 cloth-on-sphere state in contact
    on one thread."""
    import oracle
    from paper_2607_26901_amd import scenes as S
    state = S.folded_cloth_state(sc, seed=5) if "cloth_n" in sc.meta else sc
    sim = oracle.Sim(state)
    t0 = time.perf_counter()
    sim.step(iters=1)
    dt = time.perf_counter() - t0
    n_dyn = int(np.count_nonzero(sc.inv_mass > 0))
    threads = oracle.num_threads()
    # single thread, small state: 32x32 cloth after 9 oracle steps (sphere contact)
    c0 = S.c0()
    warm = oracle.Sim(c0)
    for _ in range(9):
        warm.step()
    oracle.set_num_threads(1)
    try:
        s1 = oracle.Sim(c0.with_state(x=warm.x.astype(np.float32), v=warm.v.astype(np.float32)))
        t1 = time.perf_counter()
        s1.step(iters=1)
        dt1 = time.perf_counter() - t1
    finally:
        oracle.set_num_threads(threads)
    return {"value": n_dyn / dt, "unit": "vertex-updates/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": (f"one solver iteration (brute-force candidates, Alg. 3 regions, stretch pass, Alg. 2 "
                       f"projection) over all {n_dyn} dynamic vertices of the workload's mesh in a folded "
                       f"contact state, FP64, {threads} threads, {dt:.1f} s"),
            "c0_single_thread": {"value": c0.n_dynamic / dt1, "unit": "vertex-updates/s", "cores": 1,
                                 "sample": f"one iteration of the 32x32 cloth in sphere contact, {dt1:.2f} s"}}


def run_served(args, seq_stride=1):
    """The mixed request stream (C4) served by the continuous-batching loop,
    then the same requests one mesh at a time through the single-mesh step
    (every seq_stride-th request by arrival, to bound the time).  Returns the
    comparison."""
    import torch
    from paper_2607_26901_amd import ccfr, serve
    from paper_2607_26901_amd import scenes as S

    t = time.perf_counter()
    reqs = S.c4_requests(n_requests=args.requests)
    jobs = [serve.Job(r.rid, r.arrival, r.scene, r.scene.step.steps) for r in reqs]
    log(f"[bench] c4: {len(jobs)} requests generated in {time.perf_counter() - t:.1f} s, "
        f"{sum(j.scene.n_verts for j in jobs)} vertices in all")
    budget = int(args.budget_gib * (1 << 30))
    ctx = ccfr.Context(0)
    cap = args.served_verts_cap if args.served_verts_cap > 0 else None
    # warm-up: kernels loaded, graphs recorded once, workspace grown, on a few
    # small requests
    warm = [serve.Job(j.id, 0.0, j.scene, 2) for j in sorted(jobs, key=lambda j: j.scene.n_verts)[:4]]
    # the serving loop's stored tuner choice (TUNED), or with --tune its tuner
    # run live once 16 requests are resident, or with --no-tune the defaults
    knobs = None if (args.tune or args.no_tune) else TUNED["c4"]
    if knobs:
        ctx.set_tuning(**knobs)
    srv = serve.Server(ctx, budget, tune_at=16 if args.tune else None, step_verts_cap=cap)
    srv.run(warm)
    serve.run_sequential(ctx, warm)
    torch.cuda.synchronize()

    log("[bench] c4: batched run ...")
    bst = srv.run(jobs, keep_results=True)
    srv.close()
    seq_jobs = sorted(jobs, key=lambda j: (j.arrival, j.id))[::seq_stride]
    log(f"[bench] c4: batched {bst.makespan_s:.2f} s; sequential run of {len(seq_jobs)} requests ...")
    sst = serve.run_sequential(ctx, seq_jobs, keep_results=True)
    log(f"[bench] c4: sequential {sst.makespan_s:.2f} s")
    # same accuracy: every request's final state in the mix against its run alone
    worst = 0.0
    for j in seq_jobs:
        a, b = bst.results[j.id], sst.results[j.id]
        d = float(np.abs(a.x.astype(np.float64) - b.x.astype(np.float64)).max()) / j.scene.bbox_diag()
        worst = max(worst, d)
    bs, ss = bst.summary(), sst.summary()
    desc = (f"c4: Poisson stream (200 req/s) of {len(jobs)} drape-on-sphere cloth requests, side log-uniform "
            f"in 16..512 vertices, 30 steps each at dt 1/60 s with 10 iterations, r = xi = min(2 mm, h/4); "
            f"admission budget {args.budget_gib:g} GiB of device footprint"
            + (f", at most {cap} resident vertices per step" if cap else ""))
    return {"workload": desc, "requests": len(jobs), "vertices": int(sum(j.scene.n_verts for j in jobs)),
            "budget_bytes": budget, "step_verts_cap": cap,
            "sequential_sample": (f"every {seq_stride}th request by arrival ({len(seq_jobs)} of {len(jobs)})"
                                  if seq_stride > 1 else "all requests"),
            "knobs": dict(ctx.get_tuning(), source=("stored choice of the serving loop's tuner (bench.py --tune "
                                                   "runs it live)") if knobs else
                          ("the serving loop's tuner, live" if args.tune else "defaults")),
            "batched": bs, "sequential": ss,
            "throughput_ratio": bs["throughput"] / ss["throughput"] if ss["throughput"] else None,
            "p99_request_step_ratio": (bs["p99_request_step_ms"] / ss["p99_request_step_ms"]
                                       if ss["p99_request_step_ms"] else None),
            "max_final_diff_over_diag": worst}


def bench_served(args):
    """--workload c4: the served stream as the whole bench line."""
    sv = run_served(args, seq_stride=1)
    bs = sv["batched"]
    result = {
        "metric": METRIC,
        "value": bs["throughput"],
        "unit": "vertex-updates/s",
        "n_gpus": 1,
        "steps": bs["launched_steps"],
        "warmup": 2,
        "ms_per_step": 1000.0 * bs["makespan_s"] / max(bs["launched_steps"], 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": sv["workload"], "requests": sv["requests"], "vertices": sv["vertices"],
                   "budget_bytes": sv["budget_bytes"], "iters_per_step": 10},
        "tuning": sv["knobs"],
        "p50_step_ms": bs["p50_request_step_ms"],
        "p99_step_ms": bs["p99_request_step_ms"],
        "served": sv,
    }
    print(json.dumps(result), flush=True)
    return 0


def measure(args, name, profile=True):
    """Times K graph-replayed steps of workload `name` from its initial state
    (with the knobs of TUNED, the command line or the autotuner) and, with
    `profile`, the stage rooflines from a second pass of individual launches.
    Returns the bench record and the scene."""
    import torch
    from paper_2607_26901_amd import ccfr

    sc, desc = workload(name)
    K = args.steps if args.steps is not None else sc.step.steps
    W = args.warmup
    log(f"[bench] workload {name}: N={sc.n_verts} T={sc.n_tris} E={sc.n_edges} steps={K} warmup={W}")

    ctx = ccfr.Context(0)
    mesh = ccfr.mesh_from_scene(ctx, sc)
    x0 = torch.from_numpy(sc.x.copy()).cuda()
    v0 = torch.from_numpy(sc.v.copy()).cuda()
    x = x0.clone()
    v = v0.clone()
    sp = ccfr.make_step_params(sc.step, sc.params)

    def reset():
        x.copy_(x0)
        v.copy_(v0)

    def capacity_probe(keep_at=None):
        """Run the K steps once, growing any list that overflowed; returns the
        state after step `keep_at` of the run that fitted."""
        kept = None
        for attempt in range(4):
            reset()
            ctx.sync_status(reset=True)
            for k in range(K):
                ccfr.xpbd_step(ctx, mesh, x, v, sp)
                if args.log_steps:
                    torch.cuda.synchronize()
                    log(f"[bench] probe step {k}")
                if k + 1 == keep_at:
                    kept = (x.clone(), v.clone())
            code, info = ctx.sync_status(reset=True)
            log(f"[bench] capacity probe {attempt}: status {code} need {info['need']}")
            if code == 0:
                return kept
            if code != -2:
                raise ccfr.CcfrError(code, "capacity probe")
            ctx.grow(info)
        raise RuntimeError("capacity probe did not converge")

    # knobs: given on the command line, the ones the autotuner chose for this
    # workload (TUNED, so that repeated runs time the same configuration), the
    # defaults, or (--tune) picked by the autotuner now, on steps from the
    # middle of the run (the contact state the timed steps spend most time in)
    fixed = {k: val for k, val in (("cell_scale", args.cell_scale), ("pair_split", args.pair_split),
                                    ("pair_reuse", args.pair_reuse), ("pair_skin", args.pair_skin),
                                    ("broad_phase", args.broad_phase))
             if val is not None}
    tuning = None
    if fixed or (not args.tune and not args.no_tune and name in TUNED):
        source = "given" if fixed else "chosen by the autotuner for this workload (bench.py --tune)"
        ctx.set_tuning(**(fixed or TUNED[name]))
        capacity_probe()
        tuning = dict(ctx.get_tuning(), source=source)
    elif args.tune:
        from paper_2607_26901_amd import autotune
        mid = capacity_probe(keep_at=max(1, K // 2))
        x.copy_(mid[0])
        v.copy_(mid[1])
        tuning = autotune.tune_mesh(ctx, mesh, x, v, sp, steps=min(4, K))
        tuning["source"] = f"autotuned on {min(4, K)} steps from step {max(1, K // 2)}"
        log(f"[bench] tuning: {tuning}")
        capacity_probe()                     # list sizes for the chosen knobs
    else:
        capacity_probe()

    # warmup (the first step records the step graph)
    reset()
    for _ in range(W):
        ccfr.xpbd_step(ctx, mesh, x, v, sp)
    torch.cuda.synchronize()
    reset()
    ctx.sync_status(reset=True)

    # timed region: K graph-replayed steps from the initial state
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(K):
        ccfr.xpbd_step(ctx, mesh, x, v, sp)
        ev[k + 1].record(stream)
        if args.log_steps:
            torch.cuda.synchronize()
            log(f"[bench] timed step {k}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    code, info = ctx.sync_status(reset=False)
    if code != 0:
        raise ccfr.CcfrError(code, f"timed region (status bits {info['status_bits']})")
    step_ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(K)])
    log(f"[bench] timed: {wall:.3f} s for {K} steps")

    n_dyn = sc.n_dynamic
    iters = sc.step.iters
    # solver iterations the timed steps ran (fewer than iters per step when
    # the convergence check ends a step early)
    iters_run = int(info.get("iterations_run") or iters * K)
    updates = n_dyn * iters_run
    value = updates / wall
    tot = info["totals"]
    n_builds = max(tot[9], 1)
    n_cand_builds = max(info["candidate_builds"], 1)
    P = (tot[0] + tot[1] + tot[2] + info["total_ve"]) / n_cand_builds
    Hh = tot[3] / n_builds
    Cc = tot[8] / n_builds
    used = np.zeros(sc.n_verts, bool)
    used[sc.tris.ravel()] = True
    used[sc.edges.ravel()] = True
    n_free = int(np.count_nonzero(~used))
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "vertex-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1000.0 * wall / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": desc, "n_verts": sc.n_verts, "n_dynamic": n_dyn, "n_tris": sc.n_tris,
                   "n_edges": sc.n_edges, "iters_per_step": iters, "dt": sc.step.dt},
        "iterations_run_per_step": iters_run / K,
        "p50_step_ms": float(np.percentile(step_ms, 50)),
        "p99_step_ms": float(np.percentile(step_ms, 99)),
        "gpu_ms_per_step": float(step_ms.mean()),
        "per_iteration": {"pairs_per_candidate_build": P, "candidate_builds_per_step": n_cand_builds / K,
                          "contacts": Cc, "halfspaces": Hh,
                          "violating_vertices": tot[4] / n_builds, "halted_vertices": tot[5] / n_builds},
        "halted_fraction_of_violating": (tot[5] / tot[4]) if tot[4] else 0.0,
        "pairs_per_candidate_build_by_kind": {"vf": tot[0] / n_cand_builds, "ee": tot[1] / n_cand_builds,
                                              "vv": tot[2] / n_cand_builds,
                                              "ve": info["total_ve"] / n_cand_builds},
        "tuning": tuning if tuning is not None else dict(ctx.get_tuning(), source="default"),
    }

    # profiled pass: the same K steps as individual launches with HIP events around
    # every stage on this stream; gives the per-kernel durations of the roofline
    if profile:
        reset()
        ctx.profile_enable(True)
        ctx.sync_status(reset=True)
        stage_ms = np.zeros(6)
        stage_launches = np.zeros(6)
        for _ in range(K):
            ccfr.xpbd_step(ctx, mesh, x, v, sp)
            ms, n = ctx.profile_read()
            stage_ms += ms
            stage_launches += n
        ctx.profile_enable(False)
        code, pinfo = ctx.sync_status(reset=True)
        if code != 0:
            raise ccfr.CcfrError(code, "profiled pass")
        ptot = pinfo["totals"]
        nb = max(ptot[9], 1)
        # pairs of one candidate list (written once per build, read by every
        # iteration's narrow phase), contacts and half-spaces per iteration
        n_lists = max(pinfo["candidate_builds"], 1)
        pP, pC, pH = (ptot[0] + ptot[1] + ptot[2] + pinfo["total_ve"]) / n_lists, ptot[8] / nb, ptot[3] / nb
        result["stage_ms_per_step"] = {name: float(stage_ms[i] / K) for i, name in enumerate(ccfr.STAGES)}
        # P of the method's own box test (a build per iteration at the plain
        # pad): a standalone build at the anchor after every step of a replay
        # of the same K steps (the substep's shared builds widen their boxes
        # and hold more pairs than the method reads)
        reset()
        ctx.sync_status(reset=True)
        p_samples = []
        prm = ccfr.make_params(sc.params)
        for _ in range(K):
            ccfr.xpbd_step(ctx, mesh, x, v, sp)
            ccfr.build_candidates(ctx, mesh, x, prm)
            code, binfo = ctx.sync_status(reset=True)
            if code != 0:
                raise ccfr.CcfrError(code, "pad-only candidate build")
            p_samples.append(sum(binfo["last_counts"]) + binfo["last_ve"])
        P_method = float(np.mean(p_samples))
        n_iters = float(max(pinfo["iterations_run"], 1))
        stage_idx = {name: i for i, name in enumerate(ccfr.STAGES)}
        disp = profiled_dispatches(name, ctx.get_tuning())
        N, T, E = sc.n_verts, sc.n_tris, sc.n_edges
        stages = {}
        for stage, parts in STAGE_PARTS.items():
            ms_iter = sum(stage_ms[stage_idx[q]] for q in parts) / n_iters
            B = stage_bytes(stage, N, T, E, P_method, pH)
            ach = B / (ms_iter * 1e-3) / 1e9
            stages[stage] = {"bound": "hbm", "kernels": list(STAGE_KERNELS[stage]), "achieved": ach,
                             "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                             "traffic": stage_traffic(name, ctx.get_tuning(), stage, disp) if disp else None,
                             "us_per_iteration": ms_iter * 1e3, "algorithmic_bytes": float(B)}
        dom = max(stages, key=lambda k: stages[k]["us_per_iteration"])
        result["roofline"] = dict(stages[dom], stage=dom)
        result["stage_rooflines"] = stages
        result["byte_model"] = {"N": N, "T": T, "E": E, "P_method_per_iteration": P_method,
                                "P_widened_per_build": pP, "H_per_iteration": pH, "C_per_iteration": pC,
                                "iterations": n_iters}
        it_ms = stage_ms.sum() / n_iters
        Bit = sum(stages[k]["algorithmic_bytes"] for k in stages)
        result["iteration_roofline"] = {"bytes": float(Bit), "ms": float(it_ms),
                                        "achieved_GBs": float(Bit / (it_ms * 1e-3) / 1e9),
                                        "frac": float(Bit / (it_ms * 1e-3) / 1e9 / HBM_PEAK_GBS)}
    return result, sc


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the workload's step count)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c1")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the profiled pass (no roofline)")
    ap.add_argument("--requests", type=int, default=512, help="c4: number of requests of the stream")
    ap.add_argument("--budget-gib", type=float, default=4.0, help="c4: device-footprint budget of the server")
    ap.add_argument("--served-verts-cap", type=int, default=SERVED_VERTS_CAP,
                    help="c4: most resident vertices per batched step (0: footprint budget only)")
    ap.add_argument("--no-served", action="store_true",
                    help="leave out the served-stream comparison (c4) of the default line")
    ap.add_argument("--no-coupled", action="store_true",
                    help="leave out the coupled codimensional workload (c5) of the default line")
    ap.add_argument("--served-seq-stride", type=int, default=4,
                    help="c4 in the default line: the sequential comparison runs every n-th request")
    ap.add_argument("--no-tune", action="store_true", help="default knobs, no autotuner (c4: no tuning while serving)")
    ap.add_argument("--tune", action="store_true",
                    help="run the autotuner before the timed steps instead of using the knobs it chose for this "
                         "workload (TUNED)")
    ap.add_argument("--cell-scale", type=float, default=None, help="fixed grid cell scale (skips the tuner)")
    ap.add_argument("--pair-split", type=int, default=None, help="fixed lanes per broad-phase query (skips the tuner)")
    ap.add_argument("--pair-reuse", type=int, default=None,
                    help="fixed solver iterations per candidate build (skips the tuner)")
    ap.add_argument("--pair-skin", type=int, default=None,
                    help="candidate builds that follow the motion, widened by this many r (skips the tuner)")
    ap.add_argument("--broad-phase", type=int, default=None, choices=(0, 1),
                    help="fixed broad phase: 0 hash grid, 1 bounding-volume hierarchy (skips the tuner)")
    ap.add_argument("--log-steps", action="store_true",
                    help="log every step of the capacity probe and the timed region (slow profiler runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (scale for HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the path would shard "
              f"by spatial slabs with a halo exchange, which the library does not implement)", file=sys.stderr)
        return 2

    import torch
    from paper_2607_26901_amd import ccfr

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n}))
        return 0
    if args.workload == "c4":
        return bench_served(args)
    result, sc = measure(args, args.workload, profile=not args.no_profile)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(sc)
    if not args.no_coupled and args.workload == "c1":
        # the coupled codimensional workload (all four pair kinds) on the same
        # GPU, with its stage rooflines
        sub, _ = measure(args, "c5", profile=not args.no_profile)
        result["coupled_c5"] = {k: sub[k] for k in sub if k not in (
            "metric", "n_gpus", "warmup", "higher_is_better", "scaling", "vs_baseline", "data")}
    if not args.no_served and args.workload == "c1":
        # the batched / served form on the same GPU: the C4 stream against one
        # mesh at a time (throughput and p50/p99 request-step latency)
        result["served_c4"] = run_served(args, seq_stride=max(1, args.served_seq_stride))
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
