"""ccfr_project_displacements_noalloc (no context, no allocation: its scratch is
a file-scope device array) against ccfr_project_displacements on the same
inputs, through the C ABI: two calls in a row, the second with a smaller
input, each equal to the context entry point's result bit for bit (the same
kernels run on the same data), and the device status word reported."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _regions(rng, sizes, reps):
    Ks = np.repeat(sizes, reps)
    n_list, d_list = [], []
    for K in Ks:
        n = rng.normal(size=(K, 3))
        n /= np.maximum(np.linalg.norm(n, axis=1, keepdims=True), 1e-12)
        d = rng.uniform(0, 2e-3, K)
        if K >= 4:                       # an exact duplicate
            n[1], d[1] = n[0], d[0]
        n_list.append(n)
        d_list.append(d)
    off = np.zeros(len(Ks) + 1, np.int64)
    off[1:] = np.cumsum(Ks)
    return Ks, off, n_list, d_list


def _run(ccfr, torch, ctx, off, n_list, d_list, y, w, prm):
    nh = int(off[-1])
    hs = np.zeros(max(nh, 1), ccfr.HALFSPACE_DTYPE)
    if nh:
        hs["n"][:nh] = np.concatenate(n_list).astype(np.float32)
        hs["d"][:nh] = np.concatenate(d_list).astype(np.float32)
        hs["key"][:nh] = (np.uint64(1) << np.uint64(62)) + np.arange(nh, dtype=np.uint64)
    hs = hs[:nh] if nh else hs
    regions = ccfr.caller_regions(torch.from_numpy(off.astype(np.int32)).cuda(),
                                  torch.from_numpy(hs.view(np.uint8).copy()).cuda())
    y_t = torch.from_numpy(y).cuda()
    w_t = torch.from_numpy(w).cuda()
    N = len(w)
    out_a = torch.full_like(y_t, 7.0)
    out_b = torch.full_like(y_t, -7.0)
    h_a = torch.full((N,), 9, dtype=torch.uint8).cuda()
    h_b = torch.full((N,), 5, dtype=torch.uint8).cuda()
    status = torch.full((1,), -1, dtype=torch.int32).cuda()
    ccfr.project_displacements(ctx, regions, w_t, y_t, prm, out_a, h_a)
    ccfr.project_displacements_noalloc(regions, w_t, y_t, prm, out_b, h_b, status)
    torch.cuda.synchronize()
    code, _ = ctx.sync_status(reset=True)
    return code, out_a.cpu().numpy(), out_b.cpu().numpy(), h_a.cpu().numpy(), h_b.cpu().numpy(), int(status.item())


def test_noalloc_projection_matches_context_projection():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2607_26901_amd import ccfr
    from paper_2607_26901_amd import scenes as S
    ctx = ccfr.Context(0)
    prm = S.Params(r=4e-3, xi=1e-3)
    rng = np.random.default_rng(17)
    # first call: every projection tier (regions in registers, sorted by a
    # wavefront, sorted in the scratch array), many deferred vertices
    Ks, off, n_list, d_list = _regions(rng, [0, 1, 3, 8, 9, 40, 200, 257, 300], 40)
    N = len(Ks)
    y = (rng.normal(size=(N, 3)) * 3e-3).astype(np.float32)
    w = np.ones(N, np.float32)
    w[::17] = 0.0
    y[5, 1] = np.nan                       # a non-finite proposal: y = 0, halted, status bit
    code, ya, yb, ha, hb, st = _run(ccfr, torch, ctx, off, n_list, d_list, y, w, prm)
    assert code == -4                      # the context call reports the non-finite proposal
    assert np.array_equal(ya.view(np.uint32), yb.view(np.uint32))
    assert np.array_equal(ha, hb)
    assert st == 64
    assert hb[5] == 1 and np.all(yb[5] == 0)
    assert (ha > 0).sum() >= 1 and np.any(ya != y)
    # second call right after, smaller, finite: nothing of the first remains
    Ks2, off2, n2, d2 = _regions(rng, [2, 9, 260], 5)
    N2 = len(Ks2)
    y2 = (rng.normal(size=(N2, 3)) * 3e-3).astype(np.float32)
    w2 = np.ones(N2, np.float32)
    code, ya, yb, ha, hb, st = _run(ccfr, torch, ctx, off2, n2, d2, y2, w2, prm)
    assert code == 0 and st == 0
    assert np.array_equal(ya.view(np.uint32), yb.view(np.uint32))
    assert np.array_equal(ha, hb)
    # limits are checked before anything is enqueued
    n_big = (1 << 20) + 1
    off_big = torch.zeros(n_big + 1, dtype=torch.int32, device="cuda")
    big = ccfr.Regions(n_big, 0, off_big.data_ptr(), 0, 0)
    with pytest.raises(ccfr.CcfrError) as e:
        ccfr.project_displacements_noalloc(big, torch.zeros(n_big, device="cuda"),
                                           torch.zeros(3 * n_big, device="cuda"), prm,
                                           torch.zeros(3 * n_big, device="cuda"))
    assert e.value.code == -2
