"""The soft response, visibility weights and friction (Sec. 3.3, applyResponse
of Alg. 4) on the GPU against the oracle, through the C ABI.

Call level: the oracle's regions rounded to FP32 (with each half-space's
share) are uploaded as caller-owned regions, random proposals go through
ccfr_apply_response, and every vertex must match the oracle's response on the
same FP32 inputs within 1e-5 of the bounding-box diagonal.  Substep level: a
contact scene stepped with the response on matches the oracle's substep (when
no projection decision sat near its threshold) and stays free of
penetrations."""
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


def _with_response(sc, delta_r=0.8, compliance=1e-6, vis=0.2, mu_s=0.4, mu_k=0.3):
    r = float(sc.params.r)
    prm = replace(sc.params, delta=delta_r * r, response=True, resp_compliance=compliance, vis_width=vis * r,
                  mu_s=mu_s, mu_k=mu_k)
    return replace(sc, params=prm)


def _scenes(oracle):
    base = S.c0()
    sim = oracle.Sim(base)
    for _ in range(9):
        sim.step()
    tl = S.two_layers(n=10, seed=3)
    rng = np.random.default_rng(11)
    tl.inv_mass = (tl.inv_mass * rng.uniform(0.3, 3.0, tl.n_verts)).astype(np.float32)
    return [base.with_state(x=sim.x.astype(np.float32), name="c0_contact"), tl,
            S.two_layers(n=14, seed=8, gap=2.5e-3, shift=(0.003, 0.001)),
            S.particles_in_box(nx=5, ny=5, nz=6, seed=5), S.strand_bundle(nx=4, ny=4, seg=20, seed=9)]


@pytest.mark.parametrize("k", range(5), ids=["c0_contact", "layers_mass", "layers14", "particles", "strands"])
@pytest.mark.parametrize("vis", [0.0, 0.2])
def test_apply_response_parity(env, k, vis):
    ctx, ccfr, oracle, torch = env
    sc = _with_response(_scenes(oracle)[k], vis=vis)
    om = oracle.Mesh(sc)
    off_o, hs_o, _ = oracle.regions(om, sc.params, oracle.candidates(om, sc.params))
    hs32 = H.oracle_to_fp32(hs_o)
    _, hs_w = H.to_oracle_halfspaces(off_o, hs32)
    r32 = float(np.float32(sc.params.r))
    rng = np.random.default_rng(7 + k)
    y = (rng.normal(0.0, 0.6 * r32, sc.x.shape)).astype(np.float32)
    regions = ccfr.caller_regions(torch.from_numpy(off_o.astype(np.int32)).cuda(),
                                  torch.from_numpy(hs32.view(np.uint8) if len(hs32) else np.zeros(32, np.uint8)).cuda())
    w_t = torch.from_numpy(sc.inv_mass).cuda()
    y_t = torch.from_numpy(y).cuda()
    out = torch.empty_like(y_t)
    dt = float(np.float32(sc.step.dt))
    ccfr.apply_response(ctx, regions, w_t, y_t, ccfr.make_params(sc.params), dt, out)
    torch.cuda.synchronize()
    assert ctx.sync_status(reset=True)[0] == 0
    yg = out.cpu().numpy().astype(np.float64)
    yo = oracle.response(om, sc.params, off_o, hs_w, dt, y.astype(np.float64))
    diag = sc.bbox_diag()
    err = np.linalg.norm(yg - yo, axis=1)
    assert err.max() <= H.DTOL * diag, (err.max(), int(err.argmax()))
    moved = np.linalg.norm(yo - y, axis=1) > 1e-9
    assert moved.sum() > 0, "no vertex had an active contact: the case tests nothing"


def test_response_substep_parity_and_no_penetration(env):
    ctx, ccfr, oracle, torch = env
    sc = _with_response(S.two_layers(n=12, seed=4))
    v0 = np.zeros_like(sc.x)
    v0[sc.n_verts // 2:, 2] = -0.4
    mesh = ccfr.mesh_from_scene(ctx, sc)
    x = torch.from_numpy(sc.x.copy()).cuda()
    v = torch.from_numpy(v0.copy()).cuda()
    sp = ccfr.make_step_params(sc.step, sc.params)
    sim = oracle.Sim(sc, v=v0.astype(np.float64))
    plain = oracle.Sim(replace(sc, params=replace(sc.params, response=False)), v=v0.astype(np.float64))
    xi = float(np.float32(sc.params.xi))
    compared = 0
    for step in range(3):
        ccfr.xpbd_step(ctx, mesh, x, v, sp)
        torch.cuda.synchronize()
        code, info = ctx.sync_status(reset=True)
        assert code == 0, info
        xg = x.cpu().numpy().astype(np.float64)
        assert oracle.count_intersections(xg, sc.tris, sc.edges) == 0
        _, below = oracle.min_separation(xg, sc.inv_mass, sc.tris, sc.edges, 4 * xi, xi * (1 - 1e-3))
        assert below.sum() == 0
        if step == 0:
            sim.step()
            plain.step()
            if sim.counters[6] == 0:
                assert np.abs(xg - sim.x).max() <= H.step_tol(sc, sc.step.iters)
                compared += 1
            assert np.abs(sim.x - plain.x).max() > 1e-6      # the response changed the step
    assert compared == 1


@pytest.mark.parametrize("vis", [0.0, 0.5e-3, 2e-3])
@pytest.mark.parametrize("alpha", [0.0, 1e-6])
def test_apply_response_many_active_contacts(env, vis, alpha):
    """Vertices with 2 to 300 active contacts: regions a lane takes (up to 8,
    sorted in registers), regions a wavefront takes (9 to 256: sorted in LDS,
    weights formed in parallel) and one beyond the wavefront's LDS (walked in
    order by one lane); random normals, gaps inside the repulsion range with
    ties, several visibility widths (0: every weight 1) and compliances,
    against the oracle vertex by vertex on the same FP32 regions."""
    ctx, ccfr, oracle, torch = env
    from paper_2607_26901_amd import scenes as S
    rng = np.random.default_rng(31)
    sizes = [2, 5, 15, 16, 17, 24, 33, 40, 70, 256, 300]
    delta = 1e-3
    prm = S.Params(r=2e-3, xi=1e-3, delta=delta, response=True, resp_compliance=alpha, vis_width=vis,
                   mu_s=0.4, mu_k=0.3)
    recs, off = [], [0]
    for v, K in enumerate(sizes):
        n = rng.normal(size=(K, 3))
        n /= np.linalg.norm(n, axis=1, keepdims=True)
        share = rng.uniform(0.2, 1.0, K)
        gap = rng.uniform(0.0, 0.9 * delta, K)
        gap[K // 2:] = gap[0]                      # ties of the gap
        h = np.zeros(K, ccfr.HALFSPACE_DTYPE)
        h["n"] = n.astype(np.float32)
        h["share"] = share.astype(np.float32)
        h["d"] = (share * gap).astype(np.float32)  # d = s * gap at y = 0
        h["phi"] = h["d"] / h["share"]
        h["key"] = (np.uint64(2) << np.uint64(62)) | (np.uint64(v) << np.uint64(31)) | np.arange(K, dtype=np.uint64)
        recs.append(h)
        off.append(off[-1] + K)
    hs32 = np.concatenate(recs)
    off = np.asarray(off, np.int32)
    nv = len(sizes)
    w = rng.uniform(0.5, 2.0, nv).astype(np.float32)
    y = (rng.normal(0.0, 0.3e-3, (nv, 3))).astype(np.float32)
    regions = ccfr.caller_regions(torch.from_numpy(off).cuda(), torch.from_numpy(hs32.view(np.uint8)).cuda())
    y_t = torch.from_numpy(y).cuda()
    out = torch.empty_like(y_t)
    dt = float(np.float32(1.0 / 120.0))
    ccfr.apply_response(ctx, regions, torch.from_numpy(w).cuda(), y_t, ccfr.make_params(prm), dt, out)
    torch.cuda.synchronize()
    assert ctx.sync_status(reset=True)[0] == 0
    yg = out.cpu().numpy().astype(np.float64)
    _, hs_w = H.to_oracle_halfspaces(off, hs32)
    moved = 0
    for v in range(nv):
        yo = oracle.apply_response(prm, float(w[v]), hs_w[off[v]:off[v + 1]], dt, y[v].astype(np.float64))
        assert np.abs(yg[v] - yo).max() <= 1e-9, (v, sizes[v], yg[v], yo)
        moved += np.abs(yo - y[v]).max() > 1e-9
    assert moved >= nv // 2
