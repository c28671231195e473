"""Closed-form pins of the oracle's soft response, visibility weights and
friction (Sec. 3.3, as oracle_response.c reads it).

The response energy k/2 w_c max(0, delta - d_c)^2 is the XPBD constraint
C_c = max(0, delta - d_c) with compliance 1/k; a vertex takes its share s_c of
the pair's correction, so one XPBD update moves it by
dn = w (s_c delta - rho_c) / (w + alpha / (w_c dt^2)) along n_c, where
rho_c = n_c . y + d_c is its half-space value at the proposal and
d_c = rho_c / s_c the pair's gap beyond the offset.  Visibility:
w_c = prod_j (1 - S((d_c - d_j) / delta_v)) with the cubic smoothstep S.
Friction (Macklin et al. 2014): the tangential part t of the displacement is
removed when |t| < mu_s dn, else scaled down by min(mu_k dn / |t|, 1)."""
import numpy as np
import pytest

from paper_2607_26901_amd import scenes as S

DT = 1.0 / 60.0


def _prm(**kw):
    base = dict(r=2e-3, xi=1e-3, delta=8e-4, response=True)
    base.update(kw)
    return S.Params(**base)


def _f32(v):
    return float(np.float32(v))


def test_stiff_response_restores_the_repulsion_range(orc):
    """A static floor (s = 1), the vertex phi above the offset, pushed down by
    c: with zero compliance it ends exactly delta above the offset, and its
    tangential motion is kept when there is no friction."""
    prm = _prm(resp_compliance=0.0)
    phi, c, a = 1.0e-3, 0.7e-3, 0.3e-3
    hs = orc.make_halfspaces([[0, 0, 1]], [phi], phi=[phi], share=[1.0])
    y = orc.apply_response(prm, 1.0, hs, DT, [a, 0.0, -c])
    assert np.allclose(y, [a, 0.0, _f32(prm.delta) - phi], rtol=0, atol=1e-15)
    # out of range (d = phi - c >= delta): untouched; a static vertex: untouched
    y2 = orc.apply_response(prm, 1.0, hs, DT, [a, 0.0, -0.1e-3])
    assert np.array_equal(y2, [a, 0.0, -0.1e-3])
    assert np.array_equal(orc.apply_response(prm, 0.0, hs, DT, [a, 0.0, -c]), [a, 0.0, -c])
    # switched off
    assert np.array_equal(orc.apply_response(_prm(response=False), 1.0, hs, DT, [a, 0, -c]), [a, 0, -c])


@pytest.mark.parametrize("share", [1.0, 0.25])
def test_compliant_response_and_share(orc, share):
    """Compliance alpha and a vertex side's share s: the vertex covers
    w (s delta - rho) / (w + alpha / dt^2) of the deficit."""
    alpha, w = 2e-5, 3.0
    prm = _prm(resp_compliance=alpha)
    phi = 1.0e-3
    hs = orc.make_halfspaces([[0, 0, 1]], [share * phi], phi=[phi], share=[share])
    y0 = np.array([0.0, 0.0, -0.5e-3])
    y = orc.apply_response(prm, w, hs, DT, y0)
    rho = y0[2] + share * phi
    at = _f32(alpha) / (DT * DT)
    want = w * (share * _f32(prm.delta) - rho) / (w + at)
    assert want > 0
    assert np.allclose(y - y0, [0, 0, want], rtol=1e-12, atol=0)


def test_visibility_weights_of_two_contacts(orc):
    """Two contacts with orthogonal normals: the inner one (smaller d) keeps
    weight 1 and is applied first, the outer one is attenuated by
    1 - S((d_2 - d_1) / delta_v)."""
    alpha, w, dv = 5e-5, 2.0, 4e-4
    prm = _prm(resp_compliance=alpha, vis_width=dv)
    hs = orc.make_halfspaces([[0, 0, 1], [0, 1, 0]], [0.9e-3, 1.2e-3], phi=[0.9e-3, 1.2e-3], share=[1, 1])
    y0 = np.array([0.0, -0.6e-3, -0.6e-3])
    d1, d2 = 0.9e-3 - 0.6e-3, 1.2e-3 - 0.6e-3          # 0.3 mm and 0.6 mm, both < delta = 0.8 mm
    t = (d2 - d1) / _f32(dv)
    s = t * t * (3 - 2 * t)
    w1, w2 = 1.0, 1.0 - s
    at = _f32(alpha) / (DT * DT)
    delta = _f32(prm.delta)
    dn1 = w * (delta - d1) / (w + at / w1)
    dn2 = w * (delta - d2) / (w + at / w2)
    y = orc.apply_response(prm, w, hs, DT, y0)
    assert np.allclose(y - y0, [0, dn2, dn1], rtol=1e-12, atol=0)
    # without the visibility term both get weight 1
    y_nv = orc.apply_response(_prm(resp_compliance=alpha), w, hs, DT, y0)
    assert not np.allclose(y_nv, y, rtol=1e-9, atol=0)


def test_friction_static_and_kinetic(orc):
    """Floor contact, stiff response dn = delta - d: a tangential displacement
    below mu_s dn is removed, a larger one is reduced by mu_k dn."""
    prm_s = _prm(resp_compliance=0.0, mu_s=0.5, mu_k=0.3)
    phi, c = 1.0e-3, 0.9e-3
    hs = orc.make_halfspaces([[0, 0, 1]], [phi], phi=[phi], share=[1.0])
    delta = _f32(prm_s.delta)
    dn = delta - (phi - c)
    a_small = 0.4 * dn
    y = orc.apply_response(prm_s, 1.0, hs, DT, [a_small, 0.0, -c])
    assert np.allclose(y, [0.0, 0.0, delta - phi], rtol=0, atol=1e-15)
    a_big = 3.0 * dn
    y = orc.apply_response(prm_s, 1.0, hs, DT, [a_big, 0.0, -c])
    assert np.allclose(y, [a_big - _f32(0.3) * dn, 0.0, delta - phi], rtol=1e-12, atol=1e-18)


def test_response_step_keeps_contact_scenes_valid(orc):
    """Substeps of a contact scene with the response and friction switched on:
    no penetration, separation >= xi, every iteration's motion certified, and
    the response changes the outcome."""
    from dataclasses import replace
    sc = S.two_layers(n=10, seed=3)
    prm = replace(sc.params, delta=8e-4, response=True, resp_compliance=1e-6, vis_width=2e-4, mu_s=0.4, mu_k=0.3)
    sc_r = replace(sc, params=prm)
    v = np.zeros_like(sc.x, dtype=np.float64)
    v[sc.n_verts // 2:, 2] = -0.6
    a = orc.Sim(sc_r, v=v)
    b = orc.Sim(sc, v=v)
    xi = float(np.float32(sc.params.xi))
    for _ in range(3):
        x0 = a.x.copy()
        tr = a.step(trace=True)
        b.step()
        assert orc.count_intersections(a.x, sc.tris, sc.edges) == 0
        _, below = orc.min_separation(a.x, sc.inv_mass, sc.tris, sc.edges, 4 * xi, xi * (1 - 1e-3))
        assert below.sum() == 0
        prev = x0
        for it in range(len(tr)):
            dmin, cert, _, _ = orc.motion_check(prev, tr[it], sc.inv_mass, sc.tris, sc.edges, 0.5 * xi, 4 * xi)
            assert cert and dmin >= xi * (1 - 1e-3)
            prev = tr[it]
    assert np.abs(a.x - b.x).max() > 1e-6
