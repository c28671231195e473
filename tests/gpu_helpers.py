"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI,
run the oracle on the same FP32 inputs, and compare to the stated bar."""
import numpy as np

# FP32 regions and displacements must agree with the oracle within this
# fraction of the mesh bounding-box diagonal (and normals within NTOL).
DTOL = 1e-5
NTOL = 1e-5


def step_tol(scene, iters):
    """Tolerance of a whole substep: DTOL of the diagonal, plus the rounding of
    FP32 anchor positions (half an ulp of the largest coordinate per update, two
    updates per iteration: the projection's add and the stretch pass)."""
    ulp = np.spacing(np.float32(np.abs(scene.x).max())).astype(np.float64)
    return DTOL * scene.bbox_diag() + 2 * iters * ulp


def sorted_pairs(p):
    p = np.asarray(p, np.int64).reshape(-1, 2)
    if not len(p):
        return p
    return p[np.lexsort((p[:, 1], p[:, 0]))]


def gpu_candidates(ctx, mesh, x_t, params):
    from paper_2607_26901_amd import ccfr
    import torch
    c = ccfr.build_candidates(ctx, mesh, x_t, params)
    torch.cuda.synchronize()
    got = ccfr.read_candidates(c)          # the list lengths live in the device counters
    code, info = ctx.sync_status(reset=False)
    assert code == 0, info
    return c, got, info


def gpu_regions(ctx, mesh, x_t, cands, params):
    from paper_2607_26901_amd import ccfr
    import torch
    r = ccfr.build_regions(ctx, mesh, x_t, cands, params)
    torch.cuda.synchronize()
    code, info = ctx.sync_status(reset=True)
    assert code == 0, info
    off, hs = ccfr.read_regions(r)
    return r, off, hs, info


def compare_regions(scene, params, off_g, hs_g, off_o, hs_o, xi32, r32, verts=None):
    """Match half-spaces by (vertex, key).  Returns the number compared.
    A half-space may exist on one side only if its phi sits within DTOL*diag of 2r."""
    diag = scene.bbox_diag()
    two_r = 2.0 * r32
    verts = range(scene.n_verts) if verts is None else verts
    n_cmp = 0
    for v in verts:
        g = hs_g[off_g[v]:off_g[v + 1]]
        o = hs_o[off_o[v]:off_o[v + 1]] if off_o is not None else hs_o[v]
        gk = {int(k): i for i, k in enumerate(g["key"].tolist())}
        ok = {int(k): i for i, k in enumerate(o["key"].tolist())}
        assert len(gk) == len(g), f"duplicate keys at vertex {v}"
        for k in set(gk) | set(ok):
            if k in gk and k in ok:
                a, b = g[gk[k]], o[ok[k]]
                if b["fragile"]:
                    continue
                assert np.linalg.norm(a["n"].astype(np.float64) - b["n"]) <= NTOL, (v, k, a, b)
                assert abs(float(a["d"]) - b["d"]) <= DTOL * diag, (v, k, a, b)
                assert abs(float(a["phi"]) - b["phi"]) <= DTOL * diag, (v, k, a, b)
                n_cmp += 1
            else:
                phi = float(g[gk[k]]["phi"]) if k in gk else float(o[ok[k]]["phi"])
                assert abs(phi - two_r) <= DTOL * diag, (v, k, phi, "one-sided")
    return n_cmp


def to_oracle_halfspaces(off, hs_g_like):
    """FP32 half-spaces (HALFSPACE_DTYPE) widened exactly into the oracle's layout."""
    import oracle
    out = np.zeros(len(hs_g_like), oracle.HS_DTYPE)
    out["n"] = hs_g_like["n"].astype(np.float64)
    out["d"] = hs_g_like["d"].astype(np.float64)
    out["phi"] = hs_g_like["phi"].astype(np.float64)
    out["share"] = hs_g_like["share"].astype(np.float64)
    out["key"] = hs_g_like["key"]
    return np.asarray(off, np.int64), out


def oracle_to_fp32(hs_o):
    """The oracle's FP64 half-spaces rounded to the library's FP32 layout."""
    from paper_2607_26901_amd import ccfr
    out = np.zeros(len(hs_o), ccfr.HALFSPACE_DTYPE)
    out["n"] = hs_o["n"].astype(np.float32)
    out["d"] = hs_o["d"].astype(np.float32)
    out["phi"] = hs_o["phi"].astype(np.float32)
    out["share"] = hs_o["share"].astype(np.float32)
    out["key"] = hs_o["key"]
    return out


def match_projection(oracle, params, inv_mass, x, hv, y, yg, hg, tol):
    """Compare one GPU projection (yg, halted flag hg or None) with the oracle.

    A vertex whose decisions all sit clear of their thresholds must match the
    oracle's result.  A fragile one must match the result of one branch of its
    near-threshold decisions (each branch is what Alg. 2 returns when rounding
    flips those decisions), within the same tolerance.  Returns "stable",
    "branch", or "unresolved" when the decision tree had more branches than
    the oracle walks and none of those it walked matched."""
    yo, ho, fo = oracle.project_one(params, inv_mass, x, hv, y)
    if not fo:
        assert np.linalg.norm(yg - yo) <= tol, ("stable", yg, yo)
        assert hg is None or int(hg) == int(ho), ("stable halted", hg, ho)
        return "stable"
    outs, halts, complete = oracle.project_branches(params, inv_mass, x, hv, y)
    ok = np.linalg.norm(outs - yg[None, :], axis=1) <= tol
    if hg is not None:
        ok &= halts.astype(int) == int(hg)
    if ok.any():
        return "branch"
    assert not complete, ("no branch matches", yg, hg, outs, halts)
    return "unresolved"


def steps_with_growth(ctx, mesh, sc, v0, sp, n_steps, tries=4):
    """n_steps substeps from the scene's state; a CAPACITY status grows the
    context's lists and runs the substeps again from the start.  Returns the
    final (x, v) as numpy arrays."""
    from paper_2607_26901_amd import ccfr
    import torch
    for _ in range(tries):
        x = torch.from_numpy(sc.x.copy()).cuda()
        v = torch.from_numpy(np.asarray(v0, np.float32).copy()).cuda()
        for _ in range(n_steps):
            ccfr.xpbd_step(ctx, mesh, x, v, sp)
        torch.cuda.synchronize()
        code, info = ctx.sync_status(reset=True)
        if code == 0:
            return x.cpu().numpy(), v.cpu().numpy()
        assert code == -2, info
        ctx.grow(info)
    raise AssertionError(f"lists still overflow after {tries} growths: {info}")
