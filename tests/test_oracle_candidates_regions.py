"""Pins of the oracle's candidate pairs (Sec. 4.1 broad phase, box contract) and
regions (Alg. 3, Eq. 1-3).

Candidates: the set must agree with the FP64 box test away from rounding, be
conservative for every pair within the interaction range 2r + xi (Sec. 3.1),
and respect the pair rules (no incident pairs, no static-static pairs, sorted,
unique).

Regions: checked against independent FP64 distances and the invariants the
paper states: the zero displacement lies in every region at a valid anchor,
the two sides of a pair split the gap exactly (disjoint regions, Sec. 3.1),
the normal separates the pair, and every pair within range is present."""
import numpy as np
import pytest

from paper_2607_26901_amd import scenes as S
from tests.indep_geometry import all_pair_distances


def _scenes():
    rng = np.random.default_rng(11)
    tl = S.two_layers(n=10, seed=3)
    # non-uniform masses so the shares are not all 1/2
    tl.inv_mass = (tl.inv_mass * rng.uniform(0.3, 3.0, tl.n_verts)).astype(np.float32)
    tl.inv_mass[:5] = 0.0
    parts = S.particles_in_box(nx=4, ny=4, nz=5, seed=5)
    strands = S.strand_bundle(nx=3, ny=3, seg=12, seed=9)
    tl2 = S.two_layers(n=8, seed=4, gap=2.2e-3, shift=(0.002, 0.001))
    return [tl, parts, strands, tl2]


SCENES = _scenes()


def _box_f64(x, ids, pad):
    p = x[ids]                       # [P, k, 3]
    return p.min(1) - pad, p.max(1) + pad


@pytest.mark.parametrize("sc", SCENES, ids=lambda s: s.name)
def test_candidates_match_box_definition(orc, sc):
    m = orc.Mesh(sc)
    c = orc.candidates(m, sc.params)
    pad = float(orc.box_pad(sc.params))
    x = sc.x.astype(np.float64)
    slack = 4 * np.finfo(np.float32).eps * max(1.0, np.abs(x).max())
    allp = all_pair_distances(sc.x, sc.inv_mass, sc.tris, sc.edges)
    kinds = {"vf": (lambda p: (p[:, :1], sc.tris[p[:, 1]])),
             "ee": (lambda p: (sc.edges[p[:, 0]], sc.edges[p[:, 1]])),
             "vv": (lambda p: (p[:, :1], p[:, 1:]))}
    for kind, split in kinds.items():
        got = c[kind]
        # structure: sorted, unique, legal pairs only
        if len(got):
            assert np.all(np.diff(got[:, 0].astype(np.int64) * (1 << 31) + got[:, 1]) > 0)
        legal = {tuple(p) for p in allp[kind][0].tolist()}
        assert {tuple(p) for p in got.tolist()} <= legal
        # every legal pair: inside the set iff its FP64 boxes overlap, up to rounding
        pairs = allp[kind][0]
        if not len(pairs):
            continue
        A, B = split(pairs)
        loA, hiA = _box_f64(x, A, pad)
        loB, hiB = _box_f64(x, B, pad)
        gap = np.maximum(loA - hiB, loB - hiA).max(1)      # > 0: separated on some axis
        inset = np.zeros(len(pairs), bool)
        key = pairs[:, 0] * (1 << 31) + pairs[:, 1]
        gkey = got[:, 0].astype(np.int64) * (1 << 31) + got[:, 1]
        inset[np.isin(key, gkey)] = True
        assert np.all(inset[gap < -slack])
        assert not np.any(inset[gap > slack])


@pytest.mark.parametrize("sc", SCENES, ids=lambda s: s.name)
def test_candidates_conservative_for_range(orc, sc):
    """Every pair closer than 2r + xi (where Alg. 3 keeps it) is a candidate."""
    m = orc.Mesh(sc)
    c = orc.candidates(m, sc.params)
    allp = all_pair_distances(sc.x, sc.inv_mass, sc.tris, sc.edges)
    reach = 2 * sc.params.r + sc.params.xi
    for kind in ("vf", "ee", "vv", "ve"):
        pairs, d = allp[kind]
        need = {tuple(p) for p in pairs[d < reach].tolist()}
        got = {tuple(p) for p in c[kind].tolist()}
        assert need <= got
    assert sum(len(v) for v in c.values()) > 0


def test_candidates_tiny_hand_case(orc):
    """A vertex 2 mm over a static triangle, r = xi = 1 mm: pad = 1.5 mm + guard."""
    sc = S.assemble("tiny", [S._Mesh([[0, 0, 0], [1, 0, 0], [0, 1, 0]], [[0, 1, 2]], [0, 0, 0]),
                             S.particles_mesh(np.array([[0.2, 0.2, 0.0029], [0.2, 0.2, 0.0031]]), 1.0)],
                    S.Params(r=1e-3, xi=1e-3), S.StepParams(dt=0.01))
    c = orc.candidates(orc.Mesh(sc), sc.params)
    # 2.9 mm < 2 pad = 3.000002 mm: candidate; 3.1 mm is not
    assert c["vf"].tolist() == [[3, 0]]
    # the two particles 0.2 mm apart are a VV pair
    assert c["vv"].tolist() == [[3, 4]]
    assert len(c["ee"]) == 0


def _regions(orc, sc):
    m = orc.Mesh(sc)
    c = orc.candidates(m, sc.params)
    off, hs, ndeg = orc.regions(m, sc.params, c)
    owner = np.repeat(np.arange(sc.n_verts), np.diff(off))
    return c, off, hs, owner, ndeg


def _decode(key):
    key = np.asarray(key, np.uint64)
    kind = (key >> np.uint64(62)).astype(np.int64)
    a = ((key >> np.uint64(31)) & np.uint64((1 << 31) - 1)).astype(np.int64)
    b = (key & np.uint64((1 << 31) - 1)).astype(np.int64)
    return kind, a, b


@pytest.mark.parametrize("sc", SCENES, ids=lambda s: s.name)
def test_regions_against_independent_distances(orc, sc):
    c, off, hs, owner, ndeg = _regions(orc, sc)
    assert ndeg == 0 and len(hs) > 0
    x = sc.x.astype(np.float64)
    w = sc.inv_mass.astype(np.float64)
    p = sc.params
    kind, a, b = _decode(hs["key"])
    # unit normals, phi in range, zero displacement admissible (d >= 0 at a valid anchor)
    assert np.allclose(np.linalg.norm(hs["n"], axis=1), 1.0, atol=1e-12)
    assert np.all(hs["phi"] < 2 * float(np.float32(p.r))) and np.all(hs["d"] >= 0)
    assert np.all(w[owner] > 0)
    from tests.indep_geometry import pt_tri, seg_seg
    D = hs["phi"] + float(np.float32(p.xi))      # parameters reach both paths as FP32
    for k in (1, 2, 3):
        sel = kind == k
        if not sel.any():
            continue
        A, B, n, o, dd = a[sel], b[sel], hs["n"][sel], owner[sel], D[sel]
        if k == 1:       # VF (A vertex, B triangle)
            tv = sc.tris[B]
            ind = pt_tri(x[A], x[tv[:, 0]], x[tv[:, 1]], x[tv[:, 2]])
            assert np.allclose(ind, dd, rtol=0, atol=1e-12)
            # n points from the face to the vertex on side A, and the face vertices get -n
            on_A = o == A
            nA = np.where(on_A[:, None], n, -n)
            foot = x[A] - dd[:, None] * nA
            assert np.allclose(pt_tri(foot, x[tv[:, 0]], x[tv[:, 1]], x[tv[:, 2]]), 0, atol=1e-11)
            assert np.all(on_A | (tv == o[:, None]).any(1))
        elif k == 2:     # EE (A lower edge, B higher edge)
            ea, eb = sc.edges[A], sc.edges[B]
            ind = seg_seg(x[ea[:, 0]], x[ea[:, 1]], x[eb[:, 0]], x[eb[:, 1]])
            assert np.allclose(ind, dd, rtol=0, atol=1e-12)
            on_A = (ea == o[:, None]).any(1)
            assert np.all(on_A | (eb == o[:, None]).any(1))
            nA = np.where(on_A[:, None], n, -n)
            sh = dd[:, None] * nA
            assert np.allclose(seg_seg(x[ea[:, 0]] - sh, x[ea[:, 1]] - sh, x[eb[:, 0]], x[eb[:, 1]]), 0,
                               atol=1e-11)
        else:            # VV
            assert np.allclose(np.linalg.norm(x[A] - x[B], axis=1), dd, atol=1e-12)
            on_A = o == A
            nA = np.where(on_A[:, None], n, -n)
            assert np.allclose(x[A] - x[B], dd[:, None] * nA, atol=1e-12)


@pytest.mark.parametrize("sc", SCENES, ids=lambda s: s.name)
def test_regions_share_conservation(orc, sc):
    """Eq. 2-3: the sides of a pair take shares s_A + s_B = 1 of the gap, so the
    regions of different vertices cannot overlap (Sec. 3.1): d_A + d_B = phi."""
    c, off, hs, owner, _ = _regions(orc, sc)
    x = sc.x.astype(np.float64)
    w = sc.inv_mass.astype(np.float64)
    kind, a, b = _decode(hs["key"])
    groups = {}
    for i, key in enumerate(hs["key"].tolist()):
        groups.setdefault(key, []).append(i)
    checked = 0
    for key, idx in groups.items():
        k, A, B = int(kind[idx[0]]), int(a[idx[0]]), int(b[idx[0]])
        # kinds: 0 particle-edge, 1 vertex-face, 2 edge-edge, 3 particle-particle
        sideA = [A] if k in (0, 1, 3) else list(sc.edges[A])
        sideB = list(sc.tris[B]) if k == 1 else ([B] if k == 3 else list(sc.edges[B]))
        ia = [i for i in idx if owner[i] in sideA]
        ib = [i for i in idx if owner[i] in sideB]
        assert len(ia) + len(ib) == len(idx)
        assert len(ia) == sum(w[v] > 0 for v in sideA) and len(ib) == sum(w[v] > 0 for v in sideB)
        # all vertices of a side share one half-space
        for grp in (ia, ib):
            for i in grp[1:]:
                assert np.allclose(hs["n"][i], hs["n"][grp[0]], atol=1e-14) and hs["d"][i] == hs["d"][grp[0]]
        if ia and ib:
            assert np.allclose(hs["n"][ia[0]], -hs["n"][ib[0]], atol=1e-14)
            assert np.isclose(hs["d"][ia[0]] + hs["d"][ib[0]], hs["phi"][ia[0]], rtol=1e-12, atol=1e-15)
            checked += 1
        elif ia:
            # side B static: side A takes the whole gap
            if all(w[v] == 0 for v in sideB):
                assert np.isclose(hs["d"][ia[0]], hs["phi"][ia[0]], rtol=1e-12)
    assert checked > 0 or sc.name.startswith("particles")


@pytest.mark.parametrize("sc", SCENES, ids=lambda s: s.name)
def test_regions_complete(orc, sc):
    """Every non-adjacent pair closer than 2r + xi gives each dynamic vertex with
    a non-zero share its half-space; no farther pair does."""
    c, off, hs, owner, _ = _regions(orc, sc)
    p = sc.params
    reach = 2 * p.r + p.xi
    allp = all_pair_distances(sc.x, sc.inv_mass, sc.tris, sc.edges)
    have = set(zip(owner.tolist(), hs["key"].tolist()))
    kmap = {"ve": 0, "vf": 1, "ee": 2, "vv": 3}
    w = sc.inv_mass
    for kname, (pairs, d) in allp.items():
        far = d > reach + 1e-9
        keys = (np.uint64(kmap[kname]) << np.uint64(62)) | (pairs[:, 0].astype(np.uint64) << np.uint64(31)) \
            | pairs[:, 1].astype(np.uint64)
        assert not (set(keys[far].tolist()) & set(hs["key"].tolist()))
        for (A, B), dist, key in zip(pairs[d < reach - 1e-9].tolist(), d[d < reach - 1e-9], keys[d < reach - 1e-9].tolist()):
            verts = ([A] + list(sc.tris[B])) if kname == "vf" else \
                (list(sc.edges[A]) + list(sc.edges[B]) if kname == "ee" else
                 ([A] + list(sc.edges[B]) if kname == "ve" else [A, B]))
            for v in verts:
                if w[v] > 0 and (v, key) not in have:
                    # allowed only when the pair gives this side a zero effective mass
                    assert kname == "ee"


@pytest.mark.parametrize("sc", SCENES[:2], ids=lambda s: s.name)
def test_vertex_region_bruteforce_equals_full(orc, sc):
    """The per-vertex brute-force path (used for sampled parity at full size)
    gives exactly the regions built from the full candidate lists."""
    c, off, hs, owner, _ = _regions(orc, sc)
    m = orc.Mesh(sc)
    rng = np.random.default_rng(0)
    for v in rng.choice(sc.n_verts, 40, replace=False):
        one = orc.vertex_region(m, sc.params, int(v))
        full = hs[off[v]:off[v + 1]]
        assert sorted(one["key"].tolist()) == sorted(full["key"].tolist())
        o1 = one[np.argsort(one["key"])]
        o2 = full[np.argsort(full["key"])]
        assert np.array_equal(o1["n"], o2["n"]) and np.array_equal(o1["d"], o2["d"])


def test_large_triangle_case_w2(orc):
    """W2 (Sec. 4.2 large-triangle test): a vertex over the interior of a static
    triangle whose vertices are all far outside 2r + xi still gets exactly one
    half-space n = +z, d = phi = h - xi (static face: share 1)."""
    import json, os
    table = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table5_parameters.json")))
    for name, prm in table["scenes"].items():
        r, xi = prm["r"], prm["xi"]
        h = xi + 0.5 * r
        L = 50 * (2 * r + xi)
        sc = S.assemble("w2", [S._Mesh([[-L, -L, 0], [L, -L, 0], [0, L, 0]], [[0, 1, 2]], [0, 0, 0]),
                               S.particles_mesh(np.array([[0.0, 0.0, h]]), 100.0)],
                        S.Params(r=r, xi=xi, delta=prm["delta"]), S.StepParams(dt=0.01))
        c, off, hs, owner, _ = _regions(orc, sc)
        assert len(hs) == 1 and owner[0] == 3
        hf = float(np.float32(h)) - float(np.float32(xi))
        assert np.allclose(hs["n"][0], [0, 0, 1]) and np.isclose(hs["d"][0], hf) and np.isclose(hs["phi"][0], hf)


def test_two_particles_mass_ratio_w5_w6(orc):
    """W5/W6 (Eq. 1-2): particle A may approach by s_A (D - xi), s_A = w_A/(w_A + w_B)."""
    for wa, wb in ((1.0, 1.0), (1.0, 3.0), (2.0, 0.0)):
        D, xi, r = 0.004, 0.002, 0.002
        sc = S.assemble("w5", [S.particles_mesh(np.array([[0.0, 0, 0]]), wa),
                               S.particles_mesh(np.array([[D, 0, 0]]), wb)],
                        S.Params(r=r, xi=xi), S.StepParams(dt=0.01))
        c, off, hs, owner, _ = _regions(orc, sc)
        phi = float(np.float32(D)) - float(np.float32(xi))
        assert len(hs) == (2 if wb > 0 else 1)
        i0 = np.nonzero(owner == 0)[0][0]
        assert np.allclose(hs["n"][i0], [-1, 0, 0]) and np.isclose(hs["d"][i0], wa / (wa + wb) * phi)
        if wb > 0:
            i1 = np.nonzero(owner == 1)[0][0]
            assert np.allclose(hs["n"][i1], [1, 0, 0]) and np.isclose(hs["d"][i1], wb / (wa + wb) * phi)
