"""The bounding-volume-hierarchy broad phase (tuning broad_phase = 1, the
analogue of the paper's AABB tree, Sec. 4.1) behind the same candidate
contract as the hash grid: the sorted lists equal the oracle's bit for bit on
every scene (also with boxes widened for shared builds), and whole substeps
equal the grid's bit for bit, alone and at full size."""
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
    ctx = ccfr.Context(0)
    yield ctx, ccfr, oracle, torch
    ctx.set_tuning(cell_scale=1.0, pair_split=1, pair_reuse=1, pair_skin=0, broad_phase=0)


def _scenes(oracle):
    sim = oracle.Sim(S.c0())
    for _ in range(9):
        sim.step()
    tl = S.two_layers(n=10, seed=3)
    rng = np.random.default_rng(11)
    tl.inv_mass = (tl.inv_mass * rng.uniform(0.3, 3.0, tl.n_verts)).astype(np.float32)
    tl.inv_mass[:5] = 0.0
    return {
        "c0": S.c0(),
        "c0_contact": S.c0().with_state(x=sim.x.astype(np.float32)),
        "two_layers_mass": tl,
        "two_layers14": S.two_layers(n=14, seed=8, gap=2.5e-3, shift=(0.003, 0.001)),
        "particles": S.particles_in_box(nx=5, ny=5, nz=6, seed=5),
        "strands": S.strand_bundle(nx=4, ny=4, seg=20, seed=9),
        "c1_24_folded": S.folded_cloth_state(S.c1(n=24, side=0.19), seed=3),
        "one_triangle": S.assemble("one", [S._Mesh(np.array([[0, 0, 0.0], [1e-3, 0, 0], [0, 1e-3, 0]]),
                                                   np.array([[0, 1, 2]]), [1, 1, 1])], S.Params(r=1e-3, xi=1e-3),
                                   S.StepParams(dt=1 / 60)),
    }


NAMES = ["c0", "c0_contact", "two_layers_mass", "two_layers14", "particles", "strands", "c1_24_folded",
         "one_triangle"]


@pytest.mark.parametrize("name", NAMES)
def test_lbvh_candidates_bit_exact(env, name):
    ctx, ccfr, oracle, torch = env
    sc = _scenes(oracle)[name]
    ctx.set_tuning(broad_phase=1, pair_reuse=1, pair_skin=0)
    mesh = ccfr.mesh_from_scene(ctx, sc)
    x = torch.from_numpy(sc.x.copy()).cuda()
    _, got, _ = H.gpu_candidates(ctx, mesh, x, ccfr.make_params(sc.params))
    want = oracle.candidates(oracle.Mesh(sc), sc.params)
    for k in ("vf", "ee", "vv", "ve"):
        assert np.array_equal(H.sorted_pairs(got[k]), H.sorted_pairs(want[k])), (name, k)
    ctx.set_tuning(broad_phase=0)


@pytest.mark.parametrize("name", ["c0", "two_layers14", "particles", "strands"])
@pytest.mark.parametrize("reuse,skin", [(1, 0), (3, 0), (1, 2)])
def test_lbvh_substeps_equal_grid_substeps(env, name, reuse, skin):
    """The same pairs give the same regions and the same projection: a few
    substeps are bitwise those of the grid, with builds per iteration, shared
    by three iterations, or following the motion."""
    ctx, ccfr, oracle, torch = env
    sc = _scenes(oracle)[name]
    v0 = np.zeros_like(sc.x)
    if name.startswith("two_layers"):
        v0[sc.n_verts // 2:, 2] = -0.4
    sp = ccfr.make_step_params(sc.step, sc.params)
    outs = []
    for bp in (0, 1):
        ctx.set_tuning(broad_phase=bp, pair_reuse=reuse, pair_skin=skin)
        mesh = ccfr.mesh_from_scene(ctx, sc)
        # widened boxes of shared builds can outgrow the default lists
        outs.append(H.steps_with_growth(ctx, mesh, sc, v0, sp, 3))
    ctx.set_tuning(broad_phase=0, pair_reuse=1, pair_skin=0)
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_lbvh_full_size_cloth(env):
    """The 65,536-vertex cloth in a folded state: the hierarchy's lists equal
    the grid's (bit-exact after sorting; the grid's are checked against the
    oracle by sampling in test_gpu_fullsize)."""
    ctx, ccfr, oracle, torch = env
    sc = S.c1()
    st = S.folded_cloth_state(sc, seed=5)
    lists = []
    for bp in (0, 1):
        ctx.set_tuning(broad_phase=bp, pair_reuse=1, pair_skin=0)
        mesh = ccfr.mesh_from_scene(ctx, st)
        x = torch.from_numpy(st.x.copy()).cuda()
        prm = ccfr.make_params(st.params)
        for _ in range(4):
            c = ccfr.build_candidates(ctx, mesh, x, prm)
            torch.cuda.synchronize()
            code, info = ctx.sync_status(reset=False)
            if code == 0:
                break
            assert code == -2, info
            ctx.sync_status(reset=True)
            ctx.grow(info)
        got = ccfr.read_candidates(c)
        ctx.sync_status(reset=True)
        lists.append({k: H.sorted_pairs(got[k]) for k in ("vf", "ee", "vv", "ve")})
    ctx.set_tuning(broad_phase=0)
    for k in ("vf", "ee", "vv", "ve"):
        assert np.array_equal(lists[0][k], lists[1][k]), k
    assert len(lists[0]["vf"]) > 10000 and len(lists[0]["ee"]) > 10000
