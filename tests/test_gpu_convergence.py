"""The convergence check of Alg. 4 (evaluateConvergence) and the
halting statistics on the GPU against the oracle, through the C
ABI: a substep that ends early runs the same number of iterations as the
oracle's and ends at its positions within the substep tolerance, whether it is
replayed from the recorded graph or traced; a vertex that halts every
iteration is reported with the oracle's run lengths."""
from dataclasses import replace

import numpy as np
import pytest

from paper_2607_26901_amd import scenes as S
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import oracle
    from paper_2607_26901_amd import ccfr
    return ccfr.Context(0), ccfr, oracle, torch


def _early(sc, tol_r=0.01):
    r32 = float(np.float32(sc.params.r))
    return replace(sc, step=replace(sc.step, early_exit=True, conv_tol=tol_r * r32))


def _run_gpu(ctx, ccfr, torch, sc, v0, traced=False):
    mesh = ccfr.mesh_from_scene(ctx, sc)
    x = torch.from_numpy(sc.x.copy()).cuda()
    v = torch.from_numpy(np.ascontiguousarray(v0, np.float32)).cuda()
    sp = ccfr.make_step_params(sc.step, sc.params)
    ctx.sync_status(reset=True)
    if traced:
        tr = torch.zeros((sc.step.iters, sc.n_verts, 3), dtype=torch.float32).cuda()
        ccfr.xpbd_step_traced(ctx, mesh, x, v, sp, tr)
    else:
        ccfr.xpbd_step(ctx, mesh, x, v, sp)
    torch.cuda.synchronize()
    code, info = ctx.sync_status(reset=True)
    assert code == 0, info
    return x.cpu().numpy().astype(np.float64), v.cpu().numpy().astype(np.float64), info


@pytest.mark.parametrize("case", ["free_fall", "c0_contact", "layers"])
def test_early_exit_matches_oracle(env, case):
    ctx, ccfr, oracle, torch = env
    if case == "free_fall":
        sc = S.drape(n=6, side=0.1, sphere_level=1, sphere_radius=0.05, height=0.5, jitter=1e-3, r=2e-3, xi=2e-3)
        v0 = np.zeros_like(sc.x)
        v0[:36] = [0.3, -0.1, 0.2]
    elif case == "c0_contact":
        base = S.c0()
        sim = oracle.Sim(base)
        for _ in range(9):
            sim.step()
        sc = base.with_state(x=sim.x.astype(np.float32), v=sim.v.astype(np.float32))
        v0 = sc.v
    else:
        sc = S.two_layers(n=12, seed=4)
        v0 = np.zeros_like(sc.x)
        v0[sc.n_verts // 2:, 2] = -0.3
    sc = _early(sc)
    sim = oracle.Sim(sc, v=v0.astype(np.float64))
    sim.step()
    n_it = int(sim.counters[8])
    fixed = replace(sc, step=replace(sc.step, early_exit=False, iters=n_it))
    xf, vf, _ = _run_gpu(ctx, ccfr, torch, fixed, v0)
    for traced in (False, True):
        xg, vg, info = _run_gpu(ctx, ccfr, torch, sc, v0, traced)
        # the check ends the substep where the oracle's does, and the skipped
        # iterations change nothing: the substep equals one of that many iterations
        assert info["iterations_run"] == n_it, (case, traced, info["iterations_run"], n_it)
        assert np.array_equal(xg, xf) and np.array_equal(vg, vf), (case, traced)
        # positions against the oracle when no projection decision of the
        # substep sat near its threshold (a flipped one changes the trajectory)
        if sim.counters[6] == 0:
            tol = H.step_tol(sc, n_it)
            assert np.abs(xg - sim.x).max() <= tol, (case, traced, np.abs(xg - sim.x).max(), tol)
    if case != "c0_contact":
        assert sim.counters[6] == 0
    if case == "free_fall":
        assert n_it < sc.step.iters            # the check did end the substep early


def test_early_exit_graph_replays(env):
    """Recorded-graph replays of an early-exit substep equal eager runs, over
    steps that end after different iteration counts."""
    ctx, ccfr, oracle, torch = env
    import os
    sc = _early(S.two_layers(n=10, seed=6))
    v0 = np.zeros_like(sc.x)
    v0[sc.n_verts // 2:, 2] = -0.5
    sp = ccfr.make_step_params(sc.step, sc.params)

    def run(context):
        mesh = ccfr.mesh_from_scene(context, sc)
        x = torch.from_numpy(sc.x.copy()).cuda()
        v = torch.from_numpy(v0.copy()).cuda()
        out, iters = [], []
        for _ in range(4):
            context.sync_status(reset=True)
            ccfr.xpbd_step(context, mesh, x, v, sp)
            torch.cuda.synchronize()
            _ = (x * 2).sum().item()
            out.append(x.cpu().numpy().copy())
            iters.append(context.sync_status(reset=True)[1]["iterations_run"])
        return out, iters

    os.environ["CCFR_NO_GRAPHS"] = "1"
    try:
        eager_ctx = ccfr.Context(0)
    finally:
        del os.environ["CCFR_NO_GRAPHS"]
    a, ia = run(eager_ctx)
    b, ib = run(ctx)
    assert ia == ib
    for p, q in zip(a, b):
        assert np.array_equal(p, q)


def test_halting_statistics_match_oracle(env):
    """A particle squeezed between two static triangles closer than 2 xi halts
    in every iteration: runs of 2 and of 3 or more counted as the oracle does."""
    ctx, ccfr, oracle, torch = env
    lo = S._Mesh(np.array([[-1, -1, 0.0], [1, -1, 0.0], [0, 1, 0.0]]), np.array([[0, 1, 2]]), [0, 0, 0])
    hi = S._Mesh(np.array([[-1, -1, 2.5e-3], [0, 1, 2.5e-3], [1, -1, 2.5e-3]]), np.array([[0, 1, 2]]), [0, 0, 0])
    pt = S.particles_mesh(np.array([[0.0, 0.0, 1.25e-3]]), 1.0)
    sc = S.assemble("squeeze", [lo, hi, pt], S.Params(r=1e-3, xi=1e-3, max_passes=1),
                    S.StepParams(dt=1 / 60, iters=5))
    sim = oracle.Sim(sc)
    sim.step()
    xg, vg, info = _run_gpu(ctx, ccfr, torch, sc, np.zeros_like(sc.x))
    assert info["max_halt_run"] == sim.counters[9] == 5
    assert info["halt_runs"] == [int(sim.counters[10]), int(sim.counters[11])] == [1, 3]
    assert info["iterations_run"] == 5
    assert np.array_equal(xg, sc.x.astype(np.float64))
