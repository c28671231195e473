"""Pins of the oracle's plain XPBD substep (Alg. 4) and end-to-end
checks of the property the method exists for: no interpenetration and a
separation of at least xi after every step (Sec. 4.3: zero remaining
violations at the end of every frame)."""
import numpy as np
import pytest

from paper_2607_26901_amd import scenes as S


def test_edge_coloring_valid_and_greedy(orc):
    for sc in (S.c0(), S.strand_bundle(), S.two_layers()):
        col, nc = orc.color_edges(sc.n_verts, sc.edges)
        assert nc == col.max() + 1
        seen = {}
        for e, (a, b) in enumerate(sc.edges.tolist()):
            c = col[e]
            used = seen.get(a, set()) | seen.get(b, set())
            assert c not in used                                  # colour classes share no vertex
            assert all(k in used for k in range(c))               # smallest free colour
            seen.setdefault(a, set()).add(c)
            seen.setdefault(b, set()).add(c)


def test_free_fall_closed_form(orc):
    """Far from everything and moving rigidly, each iteration moves the anchor by
    at most r towards the prediction x~ = x + dt v + dt^2 g (the clamp of Alg. 4),
    so one step moves every dynamic vertex by min(|x~ - x|, iters r) along x~ - x."""
    sc = S.drape(n=6, side=0.1, sphere_level=1, sphere_radius=0.05, height=0.5, jitter=1e-3, r=2e-3, xi=2e-3)
    sim = orc.Sim(sc)
    v0 = np.array([0.3, -0.1, 0.2])
    sim.v[:36] = v0
    x0 = sim.x.copy()
    sp = sc.step
    dt = float(np.float32(sp.dt))
    g = np.array([float(np.float32(c)) for c in sp.gravity])
    r = float(np.float32(sc.params.r))
    sim.step()
    delta = dt * v0 + dt * dt * g
    move = delta * min(1.0, sp.iters * r / np.linalg.norm(delta))
    assert np.allclose(sim.x[:36] - x0[:36], move, rtol=0, atol=1e-12)
    assert np.array_equal(sim.x[36:], x0[36:])                   # the static sphere stays
    assert np.allclose(sim.v[:36], move / dt, atol=1e-9)


def test_stiff_distance_constraint(orc):
    """With zero compliance one Gauss-Seidel pass restores a lone edge to its rest
    length, and equal masses keep its midpoint (momentum)."""
    x = np.array([[0.0, 0.0, 1.0], [0.012, 0.0, 1.0]])
    m = S._Mesh(x, np.zeros((0, 3)), [5.0, 5.0])
    m.extra_edges = np.array([[0, 1]])
    sc = S.assemble("edge", [m], S.Params(r=1.0, xi=1e-3),
                    S.StepParams(dt=1e-3, iters=1, alpha=0.0, gravity=(0, 0, 0)),
                    rest_x=np.array([[0.0, 0.0, 1.0], [0.01, 0.0, 1.0]]))
    sim = orc.Sim(sc)
    sim.step()
    assert np.isclose(np.linalg.norm(sim.x[0] - sim.x[1]), float(np.float32(0.01)), rtol=0, atol=1e-15)
    assert np.allclose(sim.x.mean(0), x.mean(0), atol=1e-15)


def test_stretch_step_conserves_linear_momentum(orc):
    """Each distance-constraint update moves its two endpoints by w_i s d and
    -w_j s d, impulses that cancel, and p restarts from the prediction every
    iteration: with no contact, no gravity and no clamped move, a step keeps the
    total momentum sum m_i v_i to rounding, whatever the masses and strains.  A
    wrong endpoint, sign or mass weighting in the pass breaks it."""
    rng = np.random.default_rng(11)
    cloth = S.cloth_grid(8, 0.16, (0.0, 0.0, 1.0))            # 20 mm edges: no self-contact
    n = len(cloth.x)
    cloth.inv_mass = rng.uniform(0.5, 2.0, n)
    cloth.v = rng.normal(0.0, 0.01, (n, 3))
    rest = cloth.x * (1.0 - 2e-4) + rng.normal(0.0, 1e-6, cloth.x.shape)   # strained by ~4 um
    sc = S.assemble("momentum", [cloth], S.Params(r=1e-4, xi=1e-4),
                    S.StepParams(dt=1e-3, iters=5, alpha=1e-7, gravity=(0.0, 0.0, 0.0)), rest_x=rest)
    sim = orc.Sim(sc)
    m = 1.0 / sim.w
    x0, v0 = sim.x.copy(), sim.v.copy()
    mom0 = (m[:, None] * v0).sum(0)
    sim.step()
    mom1 = (m[:, None] * sim.v).sum(0)
    scale = (m[:, None] * np.abs(v0)).sum(0).max()
    assert np.allclose(mom1, mom0, rtol=0, atol=1e-9 * scale), (mom0, mom1)
    # not vacuous: the pass moved the vertices away from the free prediction
    # by far more than rounding, and no move reached the clamp r
    free = x0 + float(np.float32(1e-3)) * v0
    assert np.abs(sim.x - free).max() > 1e-7
    assert np.linalg.norm(sim.x - x0, axis=1).max() < 5 * float(np.float32(1e-4))


def _check_state(orc, sc, x):
    xi = float(np.float32(sc.params.xi))
    assert orc.count_intersections(x, sc.tris, sc.edges) == 0
    dmin, below = orc.min_separation(x, sc.inv_mass, sc.tris, sc.edges, reach=4 * xi, below=xi * (1 - 1e-3))
    assert below.sum() == 0, (dmin, below)
    return dmin


def _check_motions(orc, sc, x_start, trace):
    """Every iteration's straight-line anchor motion (x before -> x after the
    iteration): certified to stay above xi / 2 (so nothing crosses), and no
    sampled distance below xi (1 - 1e-3)."""
    xi = float(np.float32(sc.params.xi))
    prev = x_start
    worst = np.inf
    for it in range(len(trace)):
        dmin, cert, ns, _ = orc.motion_check(prev, trace[it], sc.inv_mass, sc.tris, sc.edges,
                                             floor=0.5 * xi, reach=4 * xi)
        assert cert, (it, dmin, ns)
        assert dmin >= xi * (1 - 1e-3), (it, dmin)
        worst = min(worst, dmin)
        prev = trace[it]
    return worst


def test_c0_end_to_end_no_penetration(orc):
    """Config C0 (32x32 cloth onto an icosphere, 10 steps of 10 iterations): no
    interpenetration and separation >= xi after every step, and every
    iteration's motion certified free of crossings; contact starts."""
    sc = S.c0()
    sim = orc.Sim(sc)
    xi = float(np.float32(sc.params.xi))
    worst = np.inf
    for _ in range(sc.step.steps):
        x0 = sim.x.copy()
        trace = sim.step(trace=True)
        assert np.array_equal(trace[-1], sim.x)
        _check_state(orc, sc, sim.x)
        worst = min(worst, _check_motions(orc, sc, x0, trace))
    c = sim.counters
    assert c[3] > 0 and c[4] > 0              # regions were built and violated
    assert c[5] <= 0.03 * c[4] + 5             # halting stays rare (Sec. 4.3 reports <= 3%)
    assert worst < 1.5 * xi                   # the motions did come close: the check was exercised


@pytest.mark.parametrize("make", [
    lambda: S.two_layers(n=10, seed=3),
    lambda: S.strand_bundle(nx=3, ny=3, seg=12, seed=2),
    lambda: S.particles_in_box(nx=4, ny=4, nz=5, seed=6),
], ids=["two_layers", "strands", "particles"])
def test_contact_scenes_no_penetration(orc, make):
    """Scenes driven into contact: the upper layer thrown at the lower one,
    strands swung sideways into each other, particles dropped into the box."""
    sc = make()
    rng = np.random.default_rng(0)
    v = np.zeros_like(sc.x, dtype=np.float64)
    if sc.name.startswith("two_layers"):
        v[sc.n_verts // 2:, 2] = -0.6
        v += rng.normal(0, 0.05, v.shape)
    elif sc.name.startswith("bundle"):
        v[:, 0] = rng.normal(0, 0.3, sc.n_verts)
        v[:, 1] = rng.normal(0, 0.3, sc.n_verts)
    else:
        v[:, 2] = -1.0
    v[sc.inv_mass == 0] = 0
    sim = orc.Sim(sc, v=v)
    for _ in range(3):
        x0 = sim.x.copy()
        trace = sim.step(trace=True)
        _check_state(orc, sc, sim.x)
        _check_motions(orc, sc, x0, trace)
    assert sim.counters[4] > 0


def test_convergence_check_free_fall_closed_form(orc):
    """The reading of evaluateConvergence.  Far from everything, each iteration
    moves a vertex by min(|x~ - x|, r) towards the prediction; the check ends
    the step after the first iteration whose step is no longer shortened by
    the clamp, i.e. after ceil(|x~ - x| / r) iterations, at the same position
    the full iteration count reaches."""
    from dataclasses import replace
    sc = S.drape(n=6, side=0.1, sphere_level=1, sphere_radius=0.05, height=0.5, jitter=1e-3, r=2e-3, xi=2e-3)
    r = float(np.float32(sc.params.r))
    v0 = np.array([0.3, -0.1, 0.2])
    dt = float(np.float32(sc.step.dt))
    g = np.array([float(np.float32(c)) for c in sc.step.gravity])
    delta = dt * v0 + dt * dt * g
    need = int(np.ceil(np.linalg.norm(delta) / r))
    assert 1 < need < sc.step.iters
    full = orc.Sim(sc)
    full.v[:36] = v0
    full.step()
    early = orc.Sim(sc.with_state())
    early.scene = replace(sc, step=replace(sc.step, early_exit=True, conv_tol=0.01 * r))
    early.v[:36] = v0
    early.step()
    assert early.counters[8] == need and full.counters[8] == sc.step.iters
    assert np.array_equal(early.x, full.x)
    # a vertex resting on a static triangle under gravity keeps falling short:
    # the check never ends the step early
    tri = S._Mesh(np.array([[-1, -1, 0.0], [1, -1, 0.0], [0, 1, 0.0]]), np.array([[0, 1, 2]]), [0, 0, 0])
    pt = S.particles_mesh(np.array([[0.0, 0.0, 1.5e-3]]), 1.0)
    rest = S.assemble("rest", [tri, pt], S.Params(r=1e-3, xi=1e-3),
                      S.StepParams(dt=1 / 60, iters=6, early_exit=True, conv_tol=1e-5))
    sim = orc.Sim(rest)
    sim.step()
    assert sim.counters[8] == 6 and sim.counters[4] > 0


def test_consecutive_halt_statistics(orc):
    """Halting statistics: a vertex whose region cannot be satisfied within the pass
    budget halts every iteration (a run as long as the substep), one that never
    halts has none."""
    from dataclasses import replace
    # a particle squeezed between two static triangles closer than 2 xi: no
    # displacement keeps it xi from both, so every projection of a downward
    # proposal halts (max_passes = 1 leaves no verification pass)
    lo = S._Mesh(np.array([[-1, -1, 0.0], [1, -1, 0.0], [0, 1, 0.0]]), np.array([[0, 1, 2]]), [0, 0, 0])
    hi = S._Mesh(np.array([[-1, -1, 2.5e-3], [0, 1, 2.5e-3], [1, -1, 2.5e-3]]), np.array([[0, 1, 2]]), [0, 0, 0])
    pt = S.particles_mesh(np.array([[0.0, 0.0, 1.25e-3]]), 1.0)
    sc = S.assemble("squeeze", [lo, hi, pt], S.Params(r=1e-3, xi=1e-3, max_passes=1),
                    S.StepParams(dt=1 / 60, iters=5))
    sim = orc.Sim(sc)
    sim.step()
    c = sim.counters
    assert c[5] == 5 and c[9] == 5 and c[10] == 1 and c[11] == 3
    assert np.array_equal(sim.x, sc.x.astype(np.float64))        # halted every time: never moved


def test_coupled_scene_steps_stay_valid(orc):
    """The small coupled codimensional scene (rods, soft bodies with arms, a
    paper sheet, particles; all four pair kinds) through two oracle substeps:
    no penetration, every non-adjacent pair (particle-edge included) at least
    xi apart, and every iteration's straight-line motion certified."""
    sc = S.c5_small()
    sim = orc.Sim(sc)
    xi = float(np.float32(sc.params.xi))
    for step in range(2):
        prev = sim.x.copy()
        tr = sim.step(trace=True)
        assert orc.count_intersections(sim.x, sc.tris, sc.edges) == 0
        d, below = orc.min_separation(sim.x, sc.inv_mass, sc.tris, sc.edges, 4 * xi, xi * (1 - 1e-6))
        assert below.sum() == 0, (step, d, below)
        for it in range(len(tr)):
            dmin, cert, _, _ = orc.motion_check(prev, tr[it], sc.inv_mass, sc.tris, sc.edges, 0.5 * xi, 4 * xi)
            assert cert and dmin >= xi * (1 - 1e-6), (step, it, dmin)
            prev = tr[it]
    assert sim.counters[3] > 0                  # half-spaces were built
