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

value = dynamic vertices x iterations x steps / wall time of the timed region
(each update is one vertex through candidates, regions and projection in one
iteration; the stretch pass and the glue kernels are inside the timed time).
The roofline object covers the single kernel with the largest share of GPU time;
its duration is measured with HIP events on the stream in a second pass over the
same steps, run as individual launches (stage events cannot be read back from
inside a replayed graph).
cpu_baseline times the FP64 oracle on a bounded sample of the same workload.
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
    else:
        raise SystemExit(f"unknown workload {name}")
    return sc, desc


# Algorithmic bytes of one launch of each single kernel (inputs read once,
# outputs written once): N vertices, E edges, T triangles, F free particles,
# P candidate pairs, C contacts, H half-spaces of that launch.
def kernel_bytes(kernel, N, T, E, F, P, C, H):
    if kernel == "pair_emission":
        # every grid entry read once (48 B: box, index, flags, vertices): the
        # targets (triangles, edges, particles) and the vertex queries (edge
        # queries are the edge entries); free-particle flag (1 B per vertex);
        # pairs written (8 B)
        return 48 * (T + E + F + N) + N + 8 * P
    if kernel == "contacts":
        # pairs read (8 B), positions and inverse masses once (16 B/vertex), topology
        # (12 B/tri, 8 B/edge), contact records written (32 B) for the fill pass;
        # for CSR regions also the per-vertex counts (4 B/hs; inside a substep the
        # slot fill counts them instead)
        if os.environ.get("CCFR_CSR_IN_STEP") == "1":
            return 8 * P + 16 * N + 12 * T + 8 * E + 48 * C + 4 * H
        return 8 * P + 16 * N + 12 * T + 8 * E + 48 * C
    if kernel == "projection":
        # offsets (4), proposal and anchor (24), w (4), anchor written (12) per
        # vertex; half-spaces read (32 B)
        return 44 * N + 32 * H
    raise KeyError(kernel)


# Speed knobs the autotuner chose per workload (bench.py --tune, on four steps
# from the middle of the run); the default run times these.
TUNED = S_BENCH_KNOBS


# Profile summaries with counter-derived HBM traffic, per (workload, kernel).
TRAFFIC_PROFILES = {("c1", "pair_emission"): ("profiles/pair_emission_c1.md",
                                              "paper_2607_26901_amd/csrc/k_broadphase.hip"),
                    ("c1", "contacts"): ("profiles/contacts_c1.md", "paper_2607_26901_amd/csrc/k_regions.hip")}


def measured_traffic(workload, kernel, knobs):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled) from the
    committed rocprofv3 summary, or None if there is none, the kernel's source
    has changed since it was taken, or it was taken with other knobs."""
    from paper_2607_26901_amd import profiling
    entry = TRAFFIC_PROFILES.get((workload, kernel))
    if entry is None:
        return None
    summ = profiling.read_summary(os.path.join(ROOT, entry[0]))
    src = os.path.join(ROOT, entry[1])
    if "traffic_bytes_per_launch" not in summ or summ.get("source_sha256") != profiling.sha256(src):
        return None
    if summ.get("knobs") != profiling.knobs_key(knobs):
        return None
    return float(summ["traffic_bytes_per_launch"])


def cpu_baseline(sc, budget_s=25.0):
    """The oracle as it stands, one solver iteration of the whole path on the full
    mesh in a folded (contact-rich) state of the same workload."""
    import oracle
    from paper_2607_26901_amd import scenes as S
    state = S.folded_cloth_state(sc, seed=5) if "cloth_n" in sc.meta else sc
    sim = oracle.Sim(state)
    t0 = time.perf_counter()
    sim.step(iters=1)
    dt = time.perf_counter() - t0
    n_dyn = int(np.count_nonzero(sc.inv_mass > 0))
    return {"value": n_dyn / dt, "unit": "vertex-updates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": (f"one solver iteration (brute-force candidates, Alg. 3 regions, stretch pass, Alg. 2 "
                       f"projection) over all {n_dyn} dynamic vertices of the workload's mesh in a folded "
                       f"contact state, FP64, {dt:.1f} s")}


def bench_served(args):
    """The mixed request stream served by the continuous-batching loop, then the
    same stream one mesh at a time through the single-mesh step."""
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
    # warm-up: kernels loaded, graphs recorded once, workspace grown, on a few
    # small requests
    warm = [serve.Job(j.id, 0.0, j.scene, 2) for j in sorted(jobs, key=lambda j: j.scene.n_verts)[:4]]
    srv = serve.Server(ctx, budget, tune_at=None if args.no_tune else 16)
    srv.run(warm)
    serve.run_sequential(ctx, warm)
    torch.cuda.synchronize()

    log("[bench] c4: batched run ...")
    bst = srv.run(jobs, keep_results=True)
    srv.close()
    log(f"[bench] c4: batched {bst.makespan_s:.2f} s; sequential run ...")
    sst = serve.run_sequential(ctx, jobs, keep_results=True)
    log(f"[bench] c4: sequential {sst.makespan_s:.2f} s")
    # same accuracy: every request's final state in the mix against its run alone
    worst = 0.0
    for j in jobs:
        a, b = bst.results[j.id], sst.results[j.id]
        d = float(np.abs(a.x.astype(np.float64) - b.x.astype(np.float64)).max()) / j.scene.bbox_diag()
        worst = max(worst, d)
    bs, ss = bst.summary(), sst.summary()
    desc = (f"c4: Poisson stream (200 req/s) of {len(jobs)} drape-on-sphere cloth requests, side log-uniform "
            f"in 16..512 vertices, 30 steps each at dt 1/60 s with 10 iterations, r = xi = min(2 mm, h/4); "
            f"admission budget {args.budget_gib:g} GiB of device footprint")
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
        "config": {"workload": desc, "requests": len(jobs),
                   "vertices": int(sum(j.scene.n_verts for j in jobs)),
                   "budget_bytes": budget},
        "p50_step_ms": bs["p50_request_step_ms"],
        "p99_step_ms": bs["p99_request_step_ms"],
        "served": {"batched": bs, "sequential": ss,
                   "throughput_ratio": bs["throughput"] / ss["throughput"] if ss["throughput"] else None,
                   "max_final_diff_over_diag": worst},
    }
    print(json.dumps(result), flush=True)
    return 0


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
    sc, desc = workload(args.workload)
    K = args.steps if args.steps is not None else sc.step.steps
    W = args.warmup
    log(f"[bench] workload {args.workload}: N={sc.n_verts} T={sc.n_tris} E={sc.n_edges} steps={K} warmup={W}")

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
                                    ("pair_reuse", args.pair_reuse), ("pair_skin", args.pair_skin))
             if val is not None}
    tuning = None
    if fixed or (not args.tune and not args.no_tune and args.workload in TUNED):
        source = "given" if fixed else "chosen by the autotuner for this workload (bench.py --tune)"
        ctx.set_tuning(**(fixed or TUNED[args.workload]))
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
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    code, info = ctx.sync_status(reset=False)
    if code != 0:
        raise ccfr.CcfrError(code, f"timed region (status bits {info['status_bits']})")
    step_ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(K)])
    log(f"[bench] timed: {wall:.3f} s for {K} steps")

    n_dyn = sc.n_dynamic
    iters = sc.step.iters
    updates = n_dyn * iters * K
    value = updates / wall
    tot = info["totals"]
    n_builds = max(tot[9], 1)
    n_cand_builds = max(info["candidate_builds"], 1)
    P = (tot[0] + tot[1] + tot[2]) / n_cand_builds
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
        "p50_step_ms": float(np.percentile(step_ms, 50)),
        "p99_step_ms": float(np.percentile(step_ms, 99)),
        "gpu_ms_per_step": float(step_ms.mean()),
        "per_iteration": {"pairs_per_candidate_build": P, "candidate_builds_per_step": n_cand_builds / K,
                          "contacts": Cc, "halfspaces": Hh,
                          "violating_vertices": tot[4] / n_builds, "halted_vertices": tot[5] / n_builds},
        "halted_fraction_of_violating": (tot[5] / tot[4]) if tot[4] else 0.0,
        "tuning": tuning if tuning is not None else dict(ctx.get_tuning(), source="default"),
    }

    # profiled pass: the same K steps as individual launches with HIP events around
    # every stage on this stream; gives the per-kernel durations of the roofline
    if not args.no_profile:
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
        pP, pC, pH = (ptot[0] + ptot[1] + ptot[2]) / n_lists, ptot[8] / nb, ptot[3] / nb
        per_launch = stage_ms / np.maximum(stage_launches, 1)
        result["stage_ms_per_step"] = {name: float(stage_ms[i] / K) for i, name in enumerate(ccfr.STAGES)}
        # stages that are one kernel each (the projection stage is three)
        singles = {"pair_emission": 1, "contacts": 2}
        dom = max(singles, key=lambda k: stage_ms[singles[k]])
        i = singles[dom]
        B = kernel_bytes(dom, sc.n_verts, sc.n_tris, sc.n_edges, n_free, pP, pC, pH)
        if dom == "pair_emission":
            # builds that follow the motion launch the kernel every iteration and
            # it returns at once when no build is due: bytes per launch on average
            B *= n_lists / max(stage_launches[1], 1)
        achieved = B / (per_launch[i] * 1e-3) / 1e9
        result["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                              "traffic": measured_traffic(args.workload, dom, ctx.get_tuning()),
                              "avg_launch_us": float(per_launch[i] * 1e3), "algorithmic_bytes": float(B)}
        it_ms = stage_ms.sum() / max(stage_launches[5], 1)
        Bit = (60 * sc.n_verts + 24 * sc.n_tris + 16 * sc.n_edges + 8 * pP * (1 + n_lists / max(nb, 1))
               + 52 * pH)
        result["iteration_roofline"] = {"bytes": float(Bit), "ms": float(it_ms),
                                        "achieved_GBs": float(Bit / (it_ms * 1e-3) / 1e9),
                                        "frac": float(Bit / (it_ms * 1e-3) / 1e9 / HBM_PEAK_GBS)}
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(sc)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
