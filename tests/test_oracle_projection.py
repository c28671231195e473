"""Pins of the oracle's projection (Alg. 2 calling Alg. 1, the retraction and halt
fallback of Sec. 3.2, the r-ball clamp of Alg. 4).

Alg. 1 is pinned to the textbook orthogonal projection onto an affine subspace,
x0 - N^T (N N^T)^-1 (N x0 - b) (the linear-algebra background the paper cites
in Sec. 2.2).  Alg. 2 is pinned to closed-form worked cases (W1 floor slide,
W3 card stack, W4 two planes, W7 halt, W8 corner), to its invariants (the
output is admissible or the vertex halts, |y*| <= r, projecting twice equals
projecting once), and it is compared with the exact Euclidean projection onto
the region (Sec. 3.1 states the two are equivalent)."""
import itertools
import json
import os

import numpy as np
import pytest

from paper_2607_26901_amd import scenes as S

TABLE5 = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table5_parameters.json")))


def textbook_affine_projection(x0, N, b):
    N = np.atleast_2d(N)
    return x0 - N.T @ np.linalg.solve(N @ N.T, N @ x0 - b)


def _unit(v):
    return v / np.linalg.norm(v)


def test_alg1_equals_textbook_projection(orc):
    rng = np.random.default_rng(0)
    for trial in range(500):
        k = 1 + trial % 3
        N = np.stack([_unit(rng.normal(size=3)) for _ in range(k)])
        if k > 1 and np.linalg.svd(N, compute_uv=False)[-1] < 0.2:
            continue
        b = rng.normal(size=k)
        x0 = rng.normal(size=3) * 2
        st = orc.EroState()
        xt = x0.copy()
        for i in range(k):
            xt = orc.orthogonal_projection(xt, x0, N[i], b[i], st, eps=1e-12)
            ref = textbook_affine_projection(x0, N[:i + 1], b[:i + 1])
            assert np.allclose(xt, ref, atol=1e-9), (trial, i)
        assert st.m == k


def test_alg1_dependent_plane_skipped(orc):
    rng = np.random.default_rng(1)
    for _ in range(200):
        n0, n1 = _unit(rng.normal(size=3)), _unit(rng.normal(size=3))
        x0 = rng.normal(size=3)
        b0, b1 = rng.normal(size=2)
        st = orc.EroState()
        xt = orc.orthogonal_projection(x0, x0, n0, b0, st)
        xt = orc.orthogonal_projection(xt, x0, n1, b1, st)
        # a third plane that is a combination of the first two and passes through
        # their intersection is skipped, the point is unchanged
        n2 = _unit(0.3 * n0 + 0.7 * n1)
        b2 = float(np.dot(n2, xt))
        xt2 = orc.orthogonal_projection(xt, x0, n2, b2, st)
        assert st.m == 2 and np.allclose(xt2, xt, atol=1e-9)
        # a duplicate of the first plane is skipped (beta_u = 0)
        xt3 = orc.orthogonal_projection(xt, x0, n0, b0, st)
        assert st.m == 2 and np.array_equal(xt3, xt)


def test_alg1_fourth_plane_returns_unchanged(orc):
    """Alg. 1 with three planes stored: the fourth changes nothing."""
    st = orc.EroState()
    x0 = np.array([0.3, -0.2, 0.9])
    xt = x0.copy()
    for n, b in ((np.array([1., 0, 0]), 0.1), (np.array([0, 1., 0]), 0.2), (np.array([0, 0, 1.]), 0.3)):
        xt = orc.orthogonal_projection(xt, x0, n, b, st)
    assert np.allclose(xt, [0.1, 0.2, 0.3]) and st.m == 3
    xt4 = orc.orthogonal_projection(xt, x0, _unit(np.array([1., 1, 1])), 5.0, st)
    assert np.array_equal(xt4, xt) and st.m == 3


def _prm(r, xi, max_passes=4, eps=1e-6):
    return S.Params(r=r, xi=xi, max_passes=max_passes, eps_retract=eps, eps_plesnik=eps)


def _retract(y, eps):
    n = np.linalg.norm(y)
    return y * (n - eps) / n if n > eps else np.zeros(3)


def _clamp(y, r):
    n = np.linalg.norm(y)
    return y * (r / n) if n > r else y


@pytest.mark.parametrize("scene", list(TABLE5["scenes"]))
def test_w1_floor_slide(orc, scene):
    """W1 (Sec. 3.2 floor comparison): a static floor under a vertex at height h
    gives (e_z, d = h - xi); the proposal (a, 0, -c) with c > d lands on the
    plane with its tangential motion kept, shrunk by eps, then clamped to r."""
    prm = TABLE5["scenes"][scene]
    r, xi = prm["r"], prm["xi"]
    p = _prm(r, xi)
    d = 0.4 * r
    eps = float(np.float32(1e-6))
    for a, c in ((0.3 * r, 2 * d), (2.0 * r, 1.5 * d), (0.01 * r, 5 * d)):
        hs = orc.make_halfspaces([[0, 0, 1.0]], [d])
        y, h, fr = orc.project_one(p, 1.0, np.zeros(3), hs, np.array([a, 0.0, -c]))
        expect = _clamp(_retract(np.array([a, 0.0, -d]), eps), float(np.float32(r)))
        assert h == 0 and not fr
        assert np.allclose(y, expect, rtol=0, atol=1e-15)


def test_w3_card_stack_degenerate(orc):
    """W3 (Sec. 4.2 degeneration test): sheets exactly xi apart give phi = 0 and
    d = 0; a gravity proposal projects to |Delta| = 0 < eps, so y* = 0 exactly."""
    for prm in TABLE5["scenes"].values():
        p = _prm(prm["r"], prm["xi"])
        hs = orc.make_halfspaces([[0, 0, 1.0]], [0.0])
        y, h, _ = orc.project_one(p, 1.0, np.array([0.1, 0.2, 0.3]), hs, np.array([0, 0, -9.8 / 3600]))
        assert h == 0 and np.array_equal(y, np.zeros(3))


def test_w4_two_planes(orc):
    """W4 (App. A figure): two violated planes whose intersection line holds the
    Euclidean projection: the result is the textbook projection onto the line,
    shrunk by eps towards x, for angles down to near-parallel."""
    p0 = S.Params(r=1.0, xi=0.001, eps_retract=1e-15)   # retraction switched off
    eps = float(np.float32(1e-6))
    p = _prm(r=1.0, xi=0.001)
    for ang in (1.2, 0.6, 0.2, 0.05, 0.01):
        n0 = np.array([0.0, 0.0, 1.0])
        n1 = np.array([np.sin(ang), 0.0, np.cos(ang)])
        d = np.array([1e-3, 1.2e-3])
        # proposal deep inside the wedge opposite both normals: both planes are
        # active at the Euclidean projection (KKT multipliers mu > 0)
        N = np.stack([n0, n1])
        on_line = textbook_affine_projection(np.zeros(3), N, -d)
        y0 = on_line - 0.02 * n0 - 0.03 * n1 + 0.3e-3 * _unit(np.cross(n0, n1))
        line = textbook_affine_projection(y0, N, -d)
        mu = -np.linalg.solve(N @ N.T, N @ y0 + d)
        assert np.all(mu > 0)
        hs = orc.make_halfspaces(N, d)
        y, h, fr = orc.project_one(p0, 1.0, np.zeros(3), hs, y0)
        assert h == 0
        assert np.allclose(y, line, rtol=0, atol=1e-13 / np.sin(ang)), ang
        # with the retraction after each plane the result stays within O(eps)
        y, h, fr = orc.project_one(p, 1.0, np.zeros(3), hs, y0)
        assert h == 0
        assert np.linalg.norm(y - _retract(line, eps)) <= 3 * eps / np.sin(ang), ang
        assert np.all(N @ y + d >= 0)


def test_w8_corner(orc):
    """W8: three orthogonal violated planes give their corner point, then the
    eps retraction towards x, then the clamp."""
    eps = float(np.float32(1e-6))
    d = np.array([1e-3, 2e-3, 1.5e-3])
    N = np.eye(3)
    y0 = np.array([-0.01, -0.02, -0.03])
    for r in (1.0, 2e-3):
        # exact corner with the retraction switched off
        p0 = S.Params(r=r, xi=1e-3, eps_retract=1e-15)
        y, h, _ = orc.project_one(p0, 1.0, np.zeros(3), orc.make_halfspaces(N, d), y0)
        assert h == 0 and np.allclose(y, _clamp(-d, float(np.float32(r))), rtol=0, atol=1e-15)
        # retraction after each plane: within O(eps) of the retracted corner, admissible
        p = _prm(r=r, xi=1e-3)
        y, h, _ = orc.project_one(p, 1.0, np.zeros(3), orc.make_halfspaces(N, d), y0)
        expect = _clamp(_retract(-d, eps), float(np.float32(r)))
        assert h == 0 and np.linalg.norm(y - expect) <= 3 * eps and np.all(N @ y + d >= 0)


def test_w7_halt(orc):
    """W7 (Sec. 3.2): without a clean pass within max_passes the vertex falls back
    to x.  With the literal loop count 1 (the literal reading of max_passes) every violated vertex halts;
    an inconsistent set (no admissible point besides numerical noise) halts too."""
    hs = orc.make_halfspaces([[0, 0, 1.0]], [1e-3])
    y, h, _ = orc.project_one(_prm(1.0, 1e-3, max_passes=1), 1.0, np.zeros(3), hs, np.array([0, 0, -0.01]))
    assert h == 1 and np.array_equal(y, np.zeros(3))
    y, h, _ = orc.project_one(_prm(1.0, 1e-3, max_passes=2), 1.0, np.zeros(3), hs, np.array([0, 0, -0.01]))
    assert h == 0 and y[2] < 0
    # planes that only admit points near x: a cone of 5 inward planes with d = 0
    # around a proposal that is infeasible for all of them
    ang = np.linspace(0, 2 * np.pi, 6)[:-1]
    N = np.stack([[np.cos(a) * 0.6, np.sin(a) * 0.6, 0.8] for a in ang])
    y, h, _ = orc.project_one(_prm(1.0, 1e-3, max_passes=4), 1.0, np.zeros(3),
                              orc.make_halfspaces(N, np.zeros(5)), np.array([0.0, 0.0, -0.5]))
    assert np.linalg.norm(y) <= 1e-9 or h == 1
    # static vertices never move, and no region means only the clamp applies
    y, h, _ = orc.project_one(_prm(1.0, 1e-3), 0.0, np.zeros(3), hs, np.array([0, 0, -0.01]))
    assert np.array_equal(y, np.zeros(3))
    y, h, _ = orc.project_one(_prm(2e-3, 1e-3), 1.0, np.zeros(3), hs[:0], np.array([0.003, 0, -0.004]))
    assert np.allclose(y, np.array([0.003, 0, -0.004]) * float(np.float32(2e-3)) / 0.005)


def _random_region(rng, k):
    n = rng.normal(size=(k, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    d = rng.uniform(0, 2e-3, k)
    return n, d


def exact_projection(y0, N, d):
    """argmin |y - y0| s.t. N y + d >= 0, by enumerating active sets of size <= 3."""
    best, bestv = None, np.inf
    k = len(d)
    if np.all(N @ y0 + d >= -1e-15):
        return y0
    for m in (1, 2, 3):
        for act in itertools.combinations(range(k), m):
            A = N[list(act)]
            if np.linalg.matrix_rank(A, tol=1e-9) < m:
                continue
            y = textbook_affine_projection(y0, A, -d[list(act)])
            if np.all(N @ y + d >= -1e-12):
                v = np.linalg.norm(y - y0)
                if v < bestv:
                    best, bestv = y, v
    return best


def test_alg2_invariants_and_exact_projection(orc):
    """On random regions: the output is admissible (rho >= 0 for every half-space)
    unless the vertex halted to 0; |y*| <= r; projecting the output again returns
    it; and, where the paper's ordered pass reaches the region, it lands within
    the retraction margin of the exact Euclidean projection in most cases."""
    rng = np.random.default_rng(7)
    r = 4e-3
    p = _prm(r=r, xi=1e-3)
    eps = float(np.float32(1e-6))
    agree = total = 0
    for trial in range(600):
        k = 1 + trial % 6
        N, d = _random_region(rng, k)
        y0 = rng.normal(size=3) * 3e-3
        hs = orc.make_halfspaces(N, d)
        y, h, fr = orc.project_one(p, 1.0, np.zeros(3), hs, y0)
        assert np.linalg.norm(y) <= float(np.float32(r)) * (1 + 1e-12)
        if h:
            assert np.array_equal(y, np.zeros(3))
            continue
        assert np.all(N @ y + d >= -1e-15)
        y2, h2, _ = orc.project_one(p, 1.0, np.zeros(3), hs, y)
        assert h2 == 0 and np.allclose(y2, y, rtol=0, atol=1e-18)
        ex = exact_projection(y0, N, d)
        if np.linalg.norm(ex) <= r * 0.999:         # the clamp did not act
            total += 1
            agree += np.linalg.norm(y - ex) <= 10 * eps
    assert total > 100 and agree / total > 0.9, (agree, total)


def test_alg2_sort_order_and_duplicates(orc):
    """Exact duplicates do not change the result, and the result
    does not depend on the storage order of the half-spaces."""
    rng = np.random.default_rng(8)
    p = _prm(r=1.0, xi=1e-3)
    for _ in range(200):
        N, d = _random_region(rng, 5)
        y0 = rng.normal(size=3) * 3e-3
        base = orc.make_halfspaces(N, d, keys=np.arange(5) * 7)
        y, h, _ = orc.project_one(p, 1.0, np.zeros(3), base, y0)
        perm = rng.permutation(5)
        y1, h1, _ = orc.project_one(p, 1.0, np.zeros(3), base[perm], y0)
        assert h1 == h and np.array_equal(y, y1)
        dup = np.concatenate([base, base[[0, 2]]])
        dup["key"][5:] = [100, 200]
        y2, h2, _ = orc.project_one(p, 1.0, np.zeros(3), dup, y0)
        assert h2 == h and np.array_equal(y, y2)


def test_branches_of_near_threshold_decisions(orc):
    """A proposal lying exactly on a plane (rho = 0) is a decision at its
    threshold: the default branch keeps it (rho >= 0 is satisfied), the other
    treats the plane as violated, projects onto it and retracts by eps.  Both
    are results of Alg. 2 under a rounding that flips the sign; every branch is
    admissible.  A vertex with no decision near a threshold has one branch,
    equal to the plain projection."""
    prm = _prm(r=5e-3, xi=1e-3)
    x = np.zeros(3)
    hs = orc.make_halfspaces([[0, 0, 1], [1, 0, 0]], [1e-3, 2e-3])
    y = np.array([-2e-3, 0.3e-3, -1e-3])          # on plane 0, on plane 1
    outs, halts, complete = orc.project_branches(prm, 1.0, x, hs, y)
    yo, ho, fo = orc.project_one(prm, 1.0, x, hs, y)
    assert fo and complete and len(outs) >= 2
    assert np.array_equal(outs[0], yo) and halts[0] == ho
    assert np.allclose(outs[0], y, atol=0)
    # the flipped branches move the point off the planes by the retraction,
    # towards the anchor, and stay admissible
    moved = [o for o in outs if not np.array_equal(o, y)]
    assert moved
    for o in outs:
        assert np.all(hs["n"] @ o + hs["d"] >= -1e-15)
        assert np.linalg.norm(o) <= np.linalg.norm(y) + 1e-15
    y2 = np.array([0.3e-3, 0.2e-3, -3e-3])        # clearly violating plane 0 only
    outs, halts, complete = orc.project_branches(prm, 1.0, x, hs, y2)
    yo, ho, fo = orc.project_one(prm, 1.0, x, hs, y2)
    assert not fo and complete and len(outs) == 1 and np.array_equal(outs[0], yo)
