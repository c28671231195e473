"""The grid cell size changes speed only: candidates stay bit-exact with the
oracle and whole substeps give the same state for every cell scale."""
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


SCENES = {
    "two_layers": lambda: S.two_layers(n=14, seed=8, gap=2.5e-3, shift=(0.003, 0.001)),
    "particles": lambda: S.particles_in_box(nx=5, ny=5, nz=6, seed=5),
    "strands": lambda: S.strand_bundle(nx=4, ny=4, seg=20, seed=9),
}


@pytest.mark.parametrize("name", list(SCENES))
@pytest.mark.parametrize("scale,split", [(0.25, 1), (0.5, 3), (1.0, 9), (2.0, 3), (4.0, 1), (0.7, 9)])
def test_candidates_exact_at_any_cell_size(env, scale, split, name):
    ctx, ccfr, oracle, torch = env
    sc = SCENES[name]()
    ctx.set_tuning(cell_scale=scale, pair_split=split)
    try:
        mesh = ccfr.mesh_from_scene(ctx, sc)
        x = torch.from_numpy(sc.x.copy()).cuda()
        _, got, _ = H.gpu_candidates(ctx, mesh, x, ccfr.make_params(sc.params))
        want = oracle.candidates(oracle.Mesh(sc), sc.params)
        for k in ("vf", "ee", "vv", "ve"):
            assert np.array_equal(H.sorted_pairs(got[k]), H.sorted_pairs(want[k])), (k, scale)
    finally:
        ctx.set_tuning(cell_scale=1.0, pair_split=1, pair_reuse=1, pair_skin=0)


def test_steps_identical_across_cell_sizes(env):
    ctx, ccfr, oracle, torch = env
    sc = S.c0()
    sp = ccfr.make_step_params(sc.step, sc.params)
    outs = []
    for scale, split in ((1.0, 3), (0.5, 1), (1.7, 9)):
        ctx.set_tuning(cell_scale=scale, pair_split=split)
        mesh = ccfr.mesh_from_scene(ctx, sc)
        x = torch.from_numpy(sc.x.copy()).cuda()
        v = torch.from_numpy(sc.v.copy()).cuda()
        for _ in range(sc.step.steps):
            ccfr.xpbd_step(ctx, mesh, x, v, sp)
        torch.cuda.synchronize()
        code, info = ctx.sync_status(reset=True)
        assert code == 0, info
        outs.append(x.cpu().numpy())
    ctx.set_tuning(cell_scale=1.0, pair_split=1, pair_reuse=1, pair_skin=0)
    for o in outs[1:]:
        assert np.abs(o.astype(np.float64) - outs[0]).max() <= H.step_tol(sc, sc.step.iters)


def test_autotuner_picks_a_candidate_and_restores_state(env):
    ctx, ccfr, oracle, torch = env
    from paper_2607_26901_amd import autotune
    sc = S.c0()
    mesh = ccfr.mesh_from_scene(ctx, sc)
    x = torch.from_numpy(sc.x.copy()).cuda()
    v = torch.from_numpy(sc.v.copy()).cuda()
    out = autotune.tune_mesh(ctx, mesh, x, v, ccfr.make_step_params(sc.step, sc.params), steps=2,
                             candidates=(0.6, 1.0), splits=(1, 9))
    assert out["cell_scale"] in (0.6, 1.0) and out["pair_split"] in (1, 9)
    assert ctx.get_tuning()["pair_split"] == out["pair_split"]
    assert ctx.get_tuning()["cell_scale"] == pytest.approx(out["cell_scale"], rel=1e-6)
    assert np.array_equal(x.cpu().numpy(), sc.x) and np.array_equal(v.cpu().numpy(), sc.v)
    assert out["broad_phase"] in (0, 1) and ctx.get_tuning()["broad_phase"] == out["broad_phase"]
    ctx.set_tuning(cell_scale=1.0, pair_split=1, pair_reuse=1, pair_skin=0, broad_phase=0)


@pytest.mark.parametrize("name", ["c0", "two_layers", "particles", "strands", "c5_small"])
@pytest.mark.parametrize("reuse", [1, 3])
def test_direct_regions_give_the_same_substeps(env, name, reuse):
    """Slot regions written by the narrow phase itself (direct_regions) or by a
    fill launch from the contact list: the same half-spaces in another order,
    which the projection sorts, so substeps are bitwise equal; with six stretch
    colours (C0's cloth) the colours move to other host kernels and the pass
    is the same."""
    ctx, ccfr, oracle, torch = env
    sc = S.c0() if name == "c0" else S.c5_small() if name == "c5_small" else SCENES[name]()
    v0 = sc.v.copy()
    if name == "two_layers":
        v0[sc.n_verts // 2:, 2] = -0.4
    sp = ccfr.make_step_params(sc.step, sc.params)
    outs = []
    for direct in (0, 1):
        ctx.set_tuning(cell_scale=1.0, pair_split=1, pair_reuse=reuse, pair_skin=0, direct_regions=direct)
        mesh = ccfr.mesh_from_scene(ctx, sc)
        outs.append(H.steps_with_growth(ctx, mesh, sc, v0, sp, 3))
    ctx.set_tuning(cell_scale=1.0, pair_split=1, pair_reuse=1, pair_skin=0, direct_regions=0)
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
