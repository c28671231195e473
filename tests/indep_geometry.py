"""Vectorised FP64 distances for the tests, written independently of the oracle:
the minimum over a primitive pair is found by characterising where it can be
(face interior by the normal equations, or the boundary as point-segment
distances), not by the oracle's Voronoi walk."""
import numpy as np


def pt_seg(p, a, b):
    ab = b - a
    L = np.einsum("ij,ij->i", ab, ab)
    t = np.where(L > 0, np.einsum("ij,ij->i", p - a, ab) / np.where(L > 0, L, 1), 0.0)
    t = np.clip(t, 0, 1)
    return np.linalg.norm(a + t[:, None] * ab - p, axis=1)


def pt_tri(p, a, b, c):
    best = np.minimum(np.minimum(pt_seg(p, a, b), pt_seg(p, b, c)), pt_seg(p, c, a))
    ab, ac, ap = b - a, c - a, p - a
    g11 = np.einsum("ij,ij->i", ab, ab)
    g12 = np.einsum("ij,ij->i", ab, ac)
    g22 = np.einsum("ij,ij->i", ac, ac)
    r1 = np.einsum("ij,ij->i", ab, ap)
    r2 = np.einsum("ij,ij->i", ac, ap)
    det = g11 * g22 - g12 * g12
    ok = det > 1e-14 * g11 * g22
    dd = np.where(ok, det, 1)
    u = (g22 * r1 - g12 * r2) / dd
    v = (g11 * r2 - g12 * r1) / dd
    inside = ok & (u >= 0) & (v >= 0) & (u + v <= 1)
    foot = a + u[:, None] * ab + v[:, None] * ac
    df = np.linalg.norm(foot - p, axis=1)
    return np.where(inside, np.minimum(best, df), best)


def seg_seg(a, b, c, d):
    best = np.minimum(np.minimum(pt_seg(a, c, d), pt_seg(b, c, d)),
                      np.minimum(pt_seg(c, a, b), pt_seg(d, a, b)))
    u, v, w = b - a, d - c, a - c
    uu = np.einsum("ij,ij->i", u, u)
    uv = np.einsum("ij,ij->i", u, v)
    vv = np.einsum("ij,ij->i", v, v)
    uw = np.einsum("ij,ij->i", u, w)
    vw = np.einsum("ij,ij->i", v, w)
    det = uu * vv - uv * uv
    ok = det > 1e-14 * uu * vv
    dd = np.where(ok, det, 1)
    s = (uv * vw - vv * uw) / dd
    r = (uu * vw - uv * uw) / dd
    inside = ok & (s > 0) & (s < 1) & (r > 0) & (r < 1)
    q = w + s[:, None] * u - r[:, None] * v
    return np.where(inside, np.minimum(best, np.linalg.norm(q, axis=1)), best)


def pt_seg_foot(p, a, b):
    """Point-segment distance as the least of the two endpoint distances and,
    where the perpendicular foot falls strictly inside, the foot distance."""
    best = np.minimum(np.linalg.norm(p - a, axis=1), np.linalg.norm(p - b, axis=1))
    u = b - a
    uu = np.einsum("ij,ij->i", u, u)
    s = np.einsum("ij,ij->i", p - a, u) / np.where(uu > 0, uu, 1)
    inside = (uu > 0) & (s > 0) & (s < 1)
    foot = np.linalg.norm(a + s[:, None] * u - p, axis=1)
    return np.where(inside, np.minimum(best, foot), best)


def free_particles(n_verts, tris, edges):
    f = np.ones(n_verts, bool)
    f[np.asarray(tris).ravel()] = False
    f[np.asarray(edges).ravel()] = False
    return f


def all_pair_distances(x, w, tris, edges):
    """All non-adjacent, not-all-static VF, EE, free-particle VV and
    particle-edge VE pairs with their FP64 distances: dict kind -> (pairs
    [P,2], dist [P])."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    tris = np.asarray(tris, np.int64)
    edges = np.asarray(edges, np.int64)
    N, T, E = len(x), len(tris), len(edges)
    out = {}
    # VF
    if T:
        v, t = np.meshgrid(np.arange(N), np.arange(T), indexing="ij")
        v, t = v.ravel(), t.ravel()
        tv = tris[t]
        keep = (tv != v[:, None]).all(1) & ~((w[v] == 0) & (w[tv] == 0).all(1))
        v, t, tv = v[keep], t[keep], tv[keep]
        d = pt_tri(x[v], x[tv[:, 0]], x[tv[:, 1]], x[tv[:, 2]])
        out["vf"] = (np.stack([v, t], 1), d)
    else:
        out["vf"] = (np.zeros((0, 2), np.int64), np.zeros(0))
    # EE
    if E:
        i, j = np.triu_indices(E, 1)
        ei, ej = edges[i], edges[j]
        share = (ei[:, :, None] == ej[:, None, :]).any((1, 2))
        stat = (w[ei] == 0).all(1) & (w[ej] == 0).all(1)
        keep = ~share & ~stat
        i, j, ei, ej = i[keep], j[keep], ei[keep], ej[keep]
        d = seg_seg(x[ei[:, 0]], x[ei[:, 1]], x[ej[:, 0]], x[ej[:, 1]])
        out["ee"] = (np.stack([i, j], 1), d)
    else:
        out["ee"] = (np.zeros((0, 2), np.int64), np.zeros(0))
    # VV
    fr = np.nonzero(free_particles(N, tris, edges))[0]
    if len(fr) > 1:
        a, b = np.triu_indices(len(fr), 1)
        a, b = fr[a], fr[b]
        keep = ~((w[a] == 0) & (w[b] == 0))
        a, b = a[keep], b[keep]
        out["vv"] = (np.stack([a, b], 1), np.linalg.norm(x[a] - x[b], axis=1))
    else:
        out["vv"] = (np.zeros((0, 2), np.int64), np.zeros(0))
    # VE: a free particle and any edge (the particle is in no edge)
    if len(fr) and E:
        p, e = np.meshgrid(fr, np.arange(E), indexing="ij")
        p, e = p.ravel(), e.ravel()
        ev = edges[e]
        keep = ~((w[p] == 0) & (w[ev] == 0).all(1))
        p, e, ev = p[keep], e[keep], ev[keep]
        out["ve"] = (np.stack([p, e], 1), pt_seg_foot(x[p], x[ev[:, 0]], x[ev[:, 1]]))
    else:
        out["ve"] = (np.zeros((0, 2), np.int64), np.zeros(0))
    return out
