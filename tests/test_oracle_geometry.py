"""Pins of the oracle's closest-point routines (App. C: closestPointOnFace,
closestPointOnEdge) against characterisations that do not share its formulas:
the variational inequality of a projection onto a convex set, the KKT
conditions of the segment-segment minimisation, dense sampling, and textbook
special cases."""
import numpy as np
import pytest


def _rand_tri(rng):
    while True:
        t = rng.normal(0, 1, (3, 3))
        n = np.cross(t[1] - t[0], t[2] - t[0])
        if np.linalg.norm(n) > 0.05:
            return t


def test_point_triangle_variational_inequality(orc):
    """q = closest point of a convex set K to p  <=>  (p - q).(v - q) <= 0 for all v in K.
    For a triangle it suffices to check the three vertices."""
    rng = np.random.default_rng(1)
    for _ in range(3000):
        a, b, c = _rand_tri(rng)
        p = rng.normal(0, 1.5, 3)
        rc, q, bary = orc.closest_point_triangle(p, a, b, c)
        assert rc == 0
        assert np.all(bary >= -1e-12) and abs(bary.sum() - 1) < 1e-12
        assert np.allclose(q, bary @ np.stack([a, b, c]), atol=1e-12)
        for v in (a, b, c):
            assert np.dot(p - q, v - q) <= 1e-10 * (1 + np.linalg.norm(p - q) * np.linalg.norm(v - q))


def test_point_triangle_dense_sampling(orc):
    rng = np.random.default_rng(2)
    g = np.linspace(0, 1, 61)
    u, v = np.meshgrid(g, g)
    m = (u + v) <= 1
    u, v = u[m], v[m]
    for _ in range(200):
        a, b, c = _rand_tri(rng)
        p = rng.normal(0, 1.5, 3)
        _, q, _ = orc.closest_point_triangle(p, a, b, c)
        pts = a + u[:, None] * (b - a) + v[:, None] * (c - a)
        best = np.min(np.linalg.norm(pts - p, axis=1))
        assert np.linalg.norm(p - q) <= best + 1e-12


def test_point_triangle_special_cases(orc):
    a, b, c = np.array([0, 0, 0.]), np.array([1, 0, 0.]), np.array([0, 1, 0.])
    # over the interior: foot of the perpendicular
    rc, q, bary = orc.closest_point_triangle(np.array([0.2, 0.3, 0.7]), a, b, c)
    assert np.allclose(q, [0.2, 0.3, 0]) and np.allclose(bary, [0.5, 0.2, 0.3])
    # vertex region
    _, q, bary = orc.closest_point_triangle(np.array([-1, -2, 0.3]), a, b, c)
    assert np.allclose(q, a) and np.allclose(bary, [1, 0, 0])
    # edge region of the hypotenuse
    _, q, _ = orc.closest_point_triangle(np.array([1, 1, 0.]), a, b, c)
    assert np.allclose(q, [0.5, 0.5, 0])
    # degenerate (collinear) triangle
    rc, _, _ = orc.closest_point_triangle(np.array([0, 0, 1.]), a, b, 2 * b)
    assert rc == -1


def test_segments_kkt(orc):
    """For f(s,t) = |a + s d1 - c - t d2|^2 on [0,1]^2 the minimiser satisfies
    g_s = (p - q).d1 with g_s = 0 inside, >= 0 at s = 0, <= 0 at s = 1, and
    g_t = -(p - q).d2 likewise."""
    rng = np.random.default_rng(3)
    for _ in range(4000):
        a, b, c, d = rng.normal(0, 1, (4, 3))
        rc, s, t = orc.closest_points_segments(a, b, c, d)
        assert rc == 0 and 0 <= s <= 1 and 0 <= t <= 1
        p, q = a + s * (b - a), c + t * (d - c)
        gs, gt = np.dot(p - q, b - a), -np.dot(p - q, d - c)
        tol = 1e-9 * (1 + np.linalg.norm(p - q)) * 10
        for g, x in ((gs, s), (gt, t)):
            if 0 < x < 1:
                assert abs(g) < tol
            elif x == 0:
                assert g >= -tol
            else:
                assert g <= tol


def test_segments_dense_sampling(orc):
    rng = np.random.default_rng(4)
    g = np.linspace(0, 1, 201)
    for _ in range(200):
        a, b, c, d = rng.normal(0, 1, (4, 3))
        _, s, t = orc.closest_points_segments(a, b, c, d)
        dist = np.linalg.norm(a + s * (b - a) - c - t * (d - c))
        P = a + g[:, None] * (b - a)
        Q = c + g[:, None] * (d - c)
        best = np.min(np.linalg.norm(P[:, None, :] - Q[None, :, :], axis=2))
        assert dist <= best + 1e-12


def test_segments_skew_common_perpendicular(orc):
    # x-axis segment and a segment along y lifted by h: closest points are (x0,0,0), (x0,y0,h)
    rc, s, t = orc.closest_points_segments(np.array([-1, 0, 0.]), np.array([1, 0, 0.]),
                                           np.array([0.25, -1, 0.5]), np.array([0.25, 3, 0.5]))
    assert rc == 0
    assert np.isclose(-1 + 2 * s, 0.25) and np.isclose(-1 + 4 * t, 0.0)


def test_segments_parallel_rule(orc):
    """Parallel segments take the midpoint of the overlap."""
    a, b = np.array([0, 0, 0.]), np.array([1, 0, 0.])
    c, d = np.array([0.4, 0.1, 0]), np.array([1.6, 0.1, 0])
    rc, s, t = orc.closest_points_segments(a, b, c, d)
    assert rc == 1 and np.isclose(s, 0.7) and np.isclose(t, 0.25)
    # disjoint along the line: endpoint to endpoint
    rc, s, t = orc.closest_points_segments(a, b, np.array([2, 0.1, 0]), np.array([3, 0.1, 0]))
    assert rc == 1 and s == 1.0 and t == 0.0
    # zero-length edge is degenerate
    rc, _, _ = orc.closest_points_segments(a, a, c, d)
    assert rc == -1
