"""Closed-form pins of the two oracle formulas that invariants alone cannot fix.

1. Alg. 3's split of a pair's gap between its two sides when both sides are
   dynamic with unequal masses: w_side = sum_i beta_i w_i over the side's
   vertices (barycentric weights of the closest point, as printed), share
   s_A = w_A / (w_A + w_B), and every dynamic vertex of side A receives
   (n, s_A phi), of side B (-n, s_B phi) (Eq. 2 as Alg. 3 reads it).
   The geometry is dyadic so that the FP32 scene stores it exactly and the
   closest points, barycentrics and distances are known by construction; the
   masses are chosen so that a swapped share or a sum of beta^2 w gives other
   values.

2. The XPBD compliance recurrence of the stretch pass (Alg. 4):
   for a lone edge restarted from the prediction every iteration, the
   multiplier follows lambda_k = lambda* (1 - rho^k) with
   lambda* = -C / alpha~ and rho = W / (W + alpha~), so the k-th update is
   -C rho^(k-1) / (W + alpha~) and the substep ends at the prediction moved by
   the last update alone.  A missing or mis-signed alpha~ lambda term changes
   every update after the first."""
import numpy as np
import pytest

from paper_2607_26901_amd import scenes as S

H = 2.0 ** -10          # gap of the constructed pairs (about 0.98 mm)
PRM = S.Params(r=1e-3, xi=2.0 ** -11)


def _scene(x, tris, inv_mass, extra_edges=()):
    m = S._Mesh(np.asarray(x, float), np.asarray(tris, np.int64).reshape(-1, 3), inv_mass)
    m.extra_edges = np.asarray(extra_edges, np.int64).reshape(-1, 2)
    return S.assemble("shares", [m], PRM, S.StepParams(dt=1e-2, iters=1, gravity=(0, 0, 0)))


def _region(orc, sc, v):
    hs = orc.vertex_region(orc.Mesh(sc), sc.params, v)
    # the same entries from the candidate lists (the path the GPU parity uses)
    om = orc.Mesh(sc)
    off, hs_all, _ = orc.regions(om, sc.params, orc.candidates(om, sc.params))
    sub = hs_all[off[v]:off[v + 1]]
    assert sorted(sub["key"].tolist()) == sorted(hs["key"].tolist())
    return hs


def _phi():
    return H - float(np.float32(PRM.xi))


def test_vf_share_with_dynamic_face_and_interior_foot(orc):
    """Vertex p above the point with barycentrics (1/2, 1/4, 1/4) of a dynamic
    triangle; w_p = 3, w_a = 1, w_b = 2, w_c = 4, so w_f = 2 and s_p = 3/5
    (a beta^2 weighting would give w_f = 5/8, a swapped share 2/5)."""
    s = 2.0 ** -6
    x = [[0, 0, 0], [s, 0, 0], [0, s, 0], [s / 4, s / 4, H]]
    sc = _scene(x, [[0, 1, 2]], [1.0, 2.0, 4.0, 3.0])
    phi = _phi()
    hp = _region(orc, sc, 3)
    assert len(hp) == 1
    assert np.allclose(hp[0]["n"], [0, 0, 1], atol=1e-15)
    assert np.isclose(hp[0]["d"], 0.6 * phi, rtol=1e-12, atol=0)
    assert np.isclose(hp[0]["phi"], phi, rtol=1e-12, atol=0)
    for v in (0, 1, 2):
        hv = _region(orc, sc, v)
        assert len(hv) == 1 and hv[0]["key"] == hp[0]["key"]
        assert np.allclose(hv[0]["n"], [0, 0, -1], atol=1e-15)
        assert np.isclose(hv[0]["d"], 0.4 * phi, rtol=1e-12, atol=0)


def test_ve_share_particle_over_edge_interior(orc):
    """A free particle H above the point t = 1/4 of a dynamic edge (w 1 and 3:
    w_e = 3/4 + 3/4 = 3/2), w_p = 3: s_p = 2/3, the edge side 1/3 (a swapped
    share gives 1/3, a beta^2 weighting w_e = 3/4 gives 4/5).  Every vertex of
    the pair receives a half-space under the particle-edge key (kind 0)."""
    u = 2.0 ** -7
    m = S._Mesh(np.array([[-u, 0, 0], [3 * u, 0, 0], [0, 0, H]], float), np.zeros((0, 3), np.int64),
                [1.0, 3.0, 3.0])
    m.extra_edges = np.array([[0, 1]], np.int64)
    sc = S.assemble("ve_share", [m], PRM, S.StepParams(dt=1e-2, iters=1, gravity=(0, 0, 0)))
    p = int(np.nonzero(np.all(np.isclose(sc.x, [0, 0, H]), axis=1))[0][0])
    e = 0
    phi = _phi()
    key = (p << 31) | e
    hp = _region(orc, sc, p)
    assert len(hp) == 1 and int(hp[0]["key"]) == key
    assert np.allclose(hp[0]["n"], [0, 0, 1], atol=1e-15)
    assert np.isclose(hp[0]["d"], 2.0 / 3.0 * phi, rtol=1e-12, atol=0)
    assert np.isclose(hp[0]["share"], 2.0 / 3.0, rtol=1e-12, atol=0)
    for v in sc.edges[e]:
        hv = _region(orc, sc, int(v))
        assert len(hv) == 1 and int(hv[0]["key"]) == key
        assert np.allclose(hv[0]["n"], [0, 0, -1], atol=1e-15)
        assert np.isclose(hv[0]["d"], phi / 3.0, rtol=1e-12, atol=0)


def test_ve_share_particle_beyond_edge_end(orc):
    """The particle 3k behind the first endpoint and 4k above it (distance 5k):
    the foot clamps to t = 0, the normal is (-3/5, 0, 4/5) and the edge side's
    mass is its first endpoint's alone (w 1): s_p = 3/4.  The second endpoint
    carries zero weight in the split yet still receives the edge side's
    half-space (share 1/4)."""
    u, k = 2.0 ** -7, 2.0 ** -12
    m = S._Mesh(np.array([[-u, 0, 0], [3 * u, 0, 0], [-u - 3 * k, 0, 4 * k]], float), np.zeros((0, 3), np.int64),
                [1.0, 3.0, 3.0])
    m.extra_edges = np.array([[0, 1]], np.int64)
    sc = S.assemble("ve_end", [m], PRM, S.StepParams(dt=1e-2, iters=1, gravity=(0, 0, 0)))
    p = int(np.nonzero(np.all(np.isclose(sc.x, [-u - 3 * k, 0, 4 * k]), axis=1))[0][0])
    phi = 5 * k - float(np.float32(PRM.xi))
    hp = _region(orc, sc, p)
    assert len(hp) == 1
    assert np.allclose(hp[0]["n"], [-0.6, 0, 0.8], atol=1e-15)
    assert np.isclose(hp[0]["d"], 0.75 * phi, rtol=1e-12, atol=0)
    for v in sc.edges[0]:
        hv = _region(orc, sc, int(v))
        assert len(hv) == 1 and hv[0]["key"] == hp[0]["key"]
        assert np.allclose(hv[0]["n"], [0.6, 0, -0.8], atol=1e-15)
        assert np.isclose(hv[0]["d"], 0.25 * phi, rtol=1e-12, atol=0)


@pytest.mark.parametrize("active_first", [True, False], ids=["lower_index", "higher_index"])
def test_ee_share_with_interior_closest_points(orc, active_first):
    """Edge A along x with its closest point at s = 1/4 (w 1 and 3: w_A = 3/2),
    edge B along y, H above, at t = 3/4 (w 2 and 6: w_B = 5); s_A = 3/13,
    s_B = 10/13, whichever edge has the lower index."""
    u = 2.0 ** -7
    A = [[-u, 0, 0], [3 * u, 0, 0]]
    B = [[0, -3 * u, H], [0, u, H]]
    wA, wB = [1.0, 3.0], [2.0, 6.0]
    if active_first:
        x, w, ia, ib = A + B, wA + wB, (0, 1), (2, 3)
    else:
        x, w, ia, ib = B + A, wB + wA, (2, 3), (0, 1)
    sc = _scene(x, np.zeros((0, 3)), w, extra_edges=[[0, 1], [2, 3]])
    phi = _phi()
    for v in ia:
        h = _region(orc, sc, v)
        assert len(h) == 1
        assert np.allclose(h[0]["n"], [0, 0, -1], atol=1e-15)
        assert np.isclose(h[0]["d"], 3.0 / 13.0 * phi, rtol=1e-12, atol=0)
    for v in ib:
        h = _region(orc, sc, v)
        assert len(h) == 1
        assert np.allclose(h[0]["n"], [0, 0, 1], atol=1e-15)
        assert np.isclose(h[0]["d"], 10.0 / 13.0 * phi, rtol=1e-12, atol=0)


def test_fv_share_with_static_vertex(orc):
    """A static vertex q above a dynamic triangle: the face vertices take the
    whole gap (s = w_f / (w_f + 0) = 1) with n pointing from q to the face, and
    q gets no region; a static face gives the moving vertex the whole gap."""
    s = 2.0 ** -6
    x = [[0, 0, 0], [s, 0, 0], [0, s, 0], [s / 4, s / 4, H]]
    phi = _phi()
    sc = _scene(x, [[0, 1, 2]], [1.0, 2.0, 4.0, 0.0])
    assert len(_region(orc, sc, 3)) == 0
    for v in (0, 1, 2):
        h = _region(orc, sc, v)
        assert len(h) == 1
        assert np.allclose(h[0]["n"], [0, 0, -1], atol=1e-15)
        assert np.isclose(h[0]["d"], phi, rtol=1e-12, atol=0)
    sc2 = _scene(x, [[0, 1, 2]], [0.0, 0.0, 0.0, 3.0])
    h = _region(orc, sc2, 3)
    assert len(h) == 1 and np.isclose(h[0]["d"], phi, rtol=1e-12, atol=0)
    for v in (0, 1, 2):
        assert len(_region(orc, sc2, v)) == 0


@pytest.mark.parametrize("iters", [1, 2, 5])
def test_compliant_edge_multiplier_recurrence_closed_form(orc, iters):
    """A lone edge, strained by C, with alpha~ = W (rho = 1/2), no gravity and
    no velocity: after k iterations the substep ends at the prediction moved by
    the k-th update w_i dlambda_k n with dlambda_k = -C rho^(k-1) / (W + alpha~)."""
    wi, wj = 2.0, 0.5
    dt = 1e-2
    W = wi + wj
    alpha = W * dt * dt
    x = np.array([[0.0, 0.0, 1.0], [0.0125, 0.0, 1.0]])
    rest = np.array([[0.0, 0.0, 1.0], [0.01, 0.0, 1.0]])
    m = S._Mesh(x, np.zeros((0, 3)), [wi, wj])
    m.extra_edges = np.array([[0, 1]])
    sc = S.assemble("compliant_edge", [m], S.Params(r=1.0, xi=1e-3),
                    S.StepParams(dt=dt, iters=iters, alpha=alpha, gravity=(0, 0, 0)), rest_x=rest)
    sim = orc.Sim(sc)
    x0 = sim.x.copy()
    trace = sim.step(trace=True)
    dt32 = float(np.float32(dt))
    at = float(np.float32(alpha)) / (dt32 * dt32)
    xs = sc.x.astype(np.float64)
    d = xs[0] - xs[1]
    l0 = np.linalg.norm(d)
    nhat = d / l0
    L = np.linalg.norm(sc.rest_x[0].astype(np.float64) - sc.rest_x[1].astype(np.float64))
    C = l0 - L
    rho = W / (W + at)
    for k in range(1, iters + 1):
        dl = -C * rho ** (k - 1) / (W + at)
        want = np.stack([x0[0] + wi * dl * nhat, x0[1] - wj * dl * nhat])
        assert np.allclose(trace[k - 1], want, rtol=0, atol=1e-15), (k, trace[k - 1], want)
    assert np.allclose(sim.v, (sim.x - x0) / dt32, rtol=0, atol=1e-12)
    # the closed form is far from the alpha~-free update when k > 1
    if iters > 1:
        wrong = x0[0] + wi * (-C / (W + at)) * nhat
        assert np.linalg.norm(sim.x[0] - wrong) > 1e-4
