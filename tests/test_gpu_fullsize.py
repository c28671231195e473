"""Parity at the workloads' full sizes, in the benchmark's launch
configuration, on sampled outputs the oracle computes one by one.

For a sample of vertices, triangles and edges the oracle enumerates, by brute
force over the whole mesh, the candidate partners of each sampled primitive
and the region of each sampled vertex; the GPU lists and regions of the same
FP32 state must hold exactly those partners (bit-exact) and those half-spaces
(within 1e-5 of the bounding-box diagonal).  Projections of random proposals
through the GPU's regions are compared per sampled vertex.  After GPU steps of
each workload the whole state is checked for penetrations (triangle pairs by
the oracle, particle pairs by a k-d tree from scipy, strands by the oracle's
segment distances)."""
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


def _index(pairs, col):
    """Sorted view of a pair list by one column, for partner lookups."""
    p = np.asarray(pairs, np.int64).reshape(-1, 2)
    order = np.argsort(p[:, col], kind="stable")
    return p[order, col], p[order, 1 - col]


def _partners(idx, q):
    keys, other = idx
    lo, hi = np.searchsorted(keys, q, "left"), np.searchsorted(keys, q, "right")
    return np.sort(other[lo:hi])


def _sample(rng, n, k, favour=None):
    """k indices out of n: half uniform, half from `favour` (e.g. vertices with regions)."""
    out = set(rng.choice(n, size=min(k, n), replace=False).tolist())
    if favour is not None and len(favour):
        out |= set(rng.choice(favour, size=min(k, len(favour)), replace=False).tolist())
    return sorted(out)


def check_sampled(oracle, sc, x32, got, off_g, hs_g, y, yg, n_sample=48, seed=0, hg=None):
    """The CPU side: oracle queries on sampled primitives against the GPU's
    lists (`got`), regions (off_g, hs_g) and projected proposals (y -> yg)."""
    rng = np.random.default_rng(seed)
    state = sc.with_state(x=x32)
    om = oracle.Mesh(state)
    with_regions = np.nonzero(np.diff(off_g) > 0)[0]
    verts = _sample(rng, sc.n_verts, n_sample, with_regions)
    vf_by_v, vf_by_t = _index(got["vf"], 0), _index(got["vf"], 1)
    vv_a, vv_b = _index(got["vv"], 0), _index(got["vv"], 1)
    ee_a, ee_b = _index(got["ee"], 0), _index(got["ee"], 1)
    ve_p, ve_e = _index(got["ve"], 0), _index(got["ve"], 1)
    for v in verts:
        want = np.sort(oracle.vf_tris_of_vertex(om, sc.params, v))
        assert np.array_equal(_partners(vf_by_v, v), want), ("vf of vertex", v)
        want = np.sort(oracle.vv_partners_of_vertex(om, sc.params, v))
        have = np.sort(np.concatenate([_partners(vv_a, v), _partners(vv_b, v)]))
        assert np.array_equal(have, want), ("vv of vertex", v)
        want = np.sort(oracle.ve_edges_of_vertex(om, sc.params, v))
        assert np.array_equal(_partners(ve_p, v), want), ("ve of vertex", v)
    if sc.n_tris:
        for t in _sample(rng, sc.n_tris, n_sample):
            want = np.sort(oracle.vf_verts_of_tri(om, sc.params, t))
            assert np.array_equal(_partners(vf_by_t, t), want), ("vf of triangle", t)
    if sc.n_edges:
        for e in _sample(rng, sc.n_edges, n_sample):
            want = np.sort(oracle.ee_partners_of_edge(om, sc.params, e))
            have = np.sort(np.concatenate([_partners(ee_a, e), _partners(ee_b, e)]))
            assert np.array_equal(have, want), ("ee of edge", e)
            want = np.sort(oracle.ve_verts_of_edge(om, sc.params, e))
            assert np.array_equal(_partners(ve_e, e), want), ("ve of edge", e)
    # regions of the sampled vertices
    xi32, r32 = float(np.float32(sc.params.xi)), float(np.float32(sc.params.r))
    ref = {v: oracle.vertex_region(om, sc.params, v) for v in verts}
    n_cmp = H.compare_regions(state, sc.params, off_g, hs_g, None, ref, xi32, r32, verts=verts)
    # projections through the GPU's regions
    _, hs_w = H.to_oracle_halfspaces(off_g, hs_g)
    diag = state.bbox_diag()
    kinds = {"stable": 0, "branch": 0, "unresolved": 0}
    for v in verts:
        hv = hs_w[off_g[v]:off_g[v + 1]]
        # every vertex: the output lies in its region (or is the halt, zero)
        # and within r
        assert np.linalg.norm(yg[v]) <= r32 * (1 + 1e-6), v
        if len(hv):
            rho = hv["n"] @ yg[v] + hv["d"]
            assert np.all(rho >= -1e-6 * r32), (v, rho.min())
        # stable vertices match the oracle, fragile ones one branch of their
        # near-threshold decisions
        kinds[H.match_projection(oracle, sc.params, float(sc.inv_mass[v]), x32[v].astype(np.float64), hv,
                                 y[v].astype(np.float64), yg[v], None if hg is None else hg[v],
                                 H.DTOL * diag)] += 1
    print(f"{sc.name}: {len(verts)} sampled vertices, projections {kinds}, {n_cmp} half-spaces compared")
    assert kinds["stable"] + kinds["branch"] >= 0.9 * len(verts), kinds
    return len(verts), n_cmp, len(with_regions)


def sampled_parity(ctx, ccfr, oracle, torch, sc, x32, n_sample=48, seed=0, knobs=None):
    """The three calls on the GPU at state x32 (with the workload's benchmark
    knobs when given), then check_sampled."""
    x32 = np.ascontiguousarray(x32, np.float32)
    if knobs:
        ctx.set_tuning(**knobs)
    mesh = ccfr.mesh_from_scene(ctx, sc.with_state(x=x32))
    x_t = torch.from_numpy(x32).cuda()
    prm = ccfr.make_params(sc.params)
    for attempt in range(4):
        # lists sized for the default density may be too small for a folded
        # state: grow them to the reported need and build again
        c = ccfr.build_candidates(ctx, mesh, x_t, prm)
        regions = ccfr.build_regions(ctx, mesh, x_t, c, prm)
        torch.cuda.synchronize()
        code, info = ctx.sync_status(reset=False)
        if code == 0:
            break
        assert code == -2, info
        ctx.sync_status(reset=True)
        ctx.grow(info)
    else:
        raise AssertionError("capacity did not converge")
    got = ccfr.read_candidates(c)
    off_g, hs_g = ccfr.read_regions(regions)
    ctx.sync_status(reset=True)
    ctx.set_tuning(cell_scale=1.0, pair_split=1, pair_reuse=1, pair_skin=0)
    rng = np.random.default_rng(seed + 1000)
    r32 = float(np.float32(sc.params.r))
    y = (rng.normal(0.0, 1.0, (sc.n_verts, 3)) * r32).astype(np.float32)
    w_t = torch.from_numpy(sc.inv_mass).cuda()
    y_t = torch.from_numpy(y).cuda()
    out_t = torch.empty_like(y_t)
    halted_t = torch.zeros(sc.n_verts, dtype=torch.uint8).cuda()
    ccfr.project_displacements(ctx, regions, w_t, y_t, prm, out_t, halted_t)
    torch.cuda.synchronize()
    code, info = ctx.sync_status(reset=True)
    assert code == 0, info
    yg = out_t.cpu().numpy().astype(np.float64)
    return check_sampled(oracle, sc, x32, got, off_g, hs_g, y, yg, n_sample, seed, halted_t.cpu().numpy())


def run_steps(ctx, ccfr, torch, sc, steps, knobs):
    """`steps` graph-replayed substeps with the benchmark's knobs for the
    workload, as the benchmark runs them."""
    mesh = ccfr.mesh_from_scene(ctx, sc)
    x = torch.from_numpy(sc.x.copy()).cuda()
    v = torch.from_numpy(sc.v.copy()).cuda()
    sp = ccfr.make_step_params(sc.step, sc.params)
    ctx.set_tuning(**knobs)
    for _ in range(4):
        x0, v0 = x.clone(), v.clone()
        for _ in range(steps):
            ccfr.xpbd_step(ctx, mesh, x, v, sp)
        code, info = ctx.sync_status(reset=True)
        if code == 0:
            break
        assert code == -2, info
        ctx.grow(info)
        x.copy_(x0)
        v.copy_(v0)
    else:
        raise AssertionError("capacity did not converge")
    ctx.set_tuning(cell_scale=1.0, pair_split=1, pair_reuse=1, pair_skin=0)
    return x.cpu().numpy(), v.cpu().numpy()


def test_c1_folded_state(env):
    """65,536-vertex cloth in a folded, contact-rich state."""
    ctx, ccfr, oracle, torch = env
    sc = S.c1()
    st = S.folded_cloth_state(sc, seed=5)
    n, n_cmp, n_reg = sampled_parity(ctx, ccfr, oracle, torch, sc, st.x, seed=1, knobs=S.BENCH_KNOBS["c1"])
    assert n_reg > 1000 and n_cmp > 50


def test_c1_after_steps(env):
    """The 65,536-vertex cloth after 40 of its steps on the GPU (it lands at
    about step 17): no penetration, separation >= xi, and sampled parity of the
    three calls at that state."""
    ctx, ccfr, oracle, torch = env
    sc = S.c1()
    x, v = run_steps(ctx, ccfr, torch, sc, 40, S.BENCH_KNOBS["c1"])
    xg = x.astype(np.float64)
    assert oracle.count_intersections(xg, sc.tris, sc.edges) == 0
    xi = float(np.float32(sc.params.xi))
    _, below = oracle.min_separation(xg, sc.inv_mass, sc.tris, sc.edges, 4 * xi, xi * (1 - 1e-3))
    assert below.sum() == 0
    n, n_cmp, n_reg = sampled_parity(ctx, ccfr, oracle, torch, sc, x, seed=2, knobs=S.BENCH_KNOBS["c1"])
    assert n_reg > 100 and n_cmp > 10


def test_c2_strands(env):
    """650,000-vertex strands: sampled parity at the start and after 10 GPU
    steps; segment separation >= xi after them."""
    ctx, ccfr, oracle, torch = env
    sc = S.c2()
    sampled_parity(ctx, ccfr, oracle, torch, sc, sc.x, n_sample=32, seed=3, knobs=S.BENCH_KNOBS["c2"])
    x, v = run_steps(ctx, ccfr, torch, sc, 10, S.BENCH_KNOBS["c2"])
    xi = float(np.float32(sc.params.xi))
    _, below = oracle.min_separation(x.astype(np.float64), sc.inv_mass, sc.tris, sc.edges, 4 * xi,
                                     xi * (1 - 1e-3))
    assert below.sum() == 0
    sampled_parity(ctx, ccfr, oracle, torch, sc, x, n_sample=32, seed=4, knobs=S.BENCH_KNOBS["c2"])


def test_c3_particles(env):
    """2,000,000 particles in a box: sampled parity at the start and after 6 GPU
    steps; particle pairs >= xi apart (k-d tree) and inside the walls."""
    from scipy.spatial import cKDTree
    ctx, ccfr, oracle, torch = env
    sc = S.c3()
    sampled_parity(ctx, ccfr, oracle, torch, sc, sc.x, n_sample=32, seed=5, knobs=S.BENCH_KNOBS["c3"])
    x, v = run_steps(ctx, ccfr, torch, sc, 6, S.BENCH_KNOBS["c3"])
    dyn = sc.inv_mass > 0
    xi = float(np.float32(sc.params.xi))
    pairs = cKDTree(x[dyn].astype(np.float64)).query_pairs(xi * (1 - 1e-3))
    assert len(pairs) == 0
    lo = sc.x[~dyn].min(0).astype(np.float64)
    hi = sc.x[~dyn].max(0).astype(np.float64)
    xd = x[dyn].astype(np.float64)
    assert np.all(xd >= lo + xi * (1 - 1e-3)) and np.all(xd <= hi - xi * (1 - 1e-3))
    sampled_parity(ctx, ccfr, oracle, torch, sc, x, n_sample=32, seed=6, knobs=S.BENCH_KNOBS["c3"])
