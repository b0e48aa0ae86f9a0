"""Pins for the oracle's triangle-mesh obstacles (Section II-B, obstacle
term; Section II-C, targets on the collided boundary).

* closest point on a triangle: against dense barycentric sampling, and in
  each Voronoi region against its closed form;
* closest point and inside test over a mesh: against the closed-form signed
  distance of a box, and the inside test of a sphere;
* the response: targets in closed form for a box, and a finger pressed by a
  fine icosphere ends within the discretisation error of the same finger
  pressed by the analytic sphere.
"""
import dataclasses

import numpy as np
import pytest

from paper_2203_02054_amd import meshgen as mg
import oracle
from oracle.collision import MESH, SPHERE
from oracle.obstacle import EDGE, FACE, VERTEX, MeshObstacle, closest_on_triangles
from tests.meshes import pressed_finger


def test_closest_point_on_a_triangle_beats_dense_sampling():
    rng = np.random.default_rng(31)
    u = np.linspace(0, 1, 161)
    bu, bv = np.meshgrid(u, u)
    keep = bu + bv <= 1
    bu, bv = bu[keep], bv[keep]
    for _ in range(40):
        a, b, c = rng.normal(size=(3, 3, 1))
        p = rng.normal(size=3) * 2
        q, kind, loc = closest_on_triangles(p, a, b, c)
        samples = a + (b - a) * bu + (c - a) * bv
        dmin = np.sqrt(((samples - p[:, None]) ** 2).sum(axis=0)).min()
        d = np.linalg.norm(q[:, 0] - p)
        assert d <= dmin + 1e-12
        # q is on the triangle: barycentric coordinates in [0, 1]
        M = np.stack([(b - a)[:, 0], (c - a)[:, 0]], axis=1)
        lam, *_ = np.linalg.lstsq(M, q[:, 0] - a[:, 0], rcond=None)
        assert lam.min() >= -1e-10 and lam.sum() <= 1 + 1e-10
        assert np.linalg.norm(M @ lam - (q[:, 0] - a[:, 0])) < 1e-10


def test_closest_point_regions_in_closed_form():
    a, b, c = (np.array([[0.0], [0.0], [0.0]]), np.array([[2.0], [0.0], [0.0]]), np.array([[0.0], [2.0], [0.0]]))
    cases = [((0.5, 0.5, 3.0), (0.5, 0.5, 0.0), FACE, 0),
             ((-1.0, -1.0, 1.0), (0.0, 0.0, 0.0), VERTEX, 0),
             ((3.0, -0.5, -1.0), (2.0, 0.0, 0.0), VERTEX, 1),
             ((-0.5, 4.0, 2.0), (0.0, 2.0, 0.0), VERTEX, 2),
             ((1.0, -3.0, 0.5), (1.0, 0.0, 0.0), EDGE, 0),
             ((-2.0, 1.5, 0.0), (0.0, 1.5, 0.0), EDGE, 1),
             ((2.0, 2.0, 1.0), (1.0, 1.0, 0.0), EDGE, 2)]
    for p, want, kind, loc in cases:
        q, k, l = closest_on_triangles(np.array(p), a, b, c)
        np.testing.assert_allclose(q[:, 0], want, atol=1e-15)
        assert (k[0], l[0]) == (kind, loc)


def _box_sd(p, lo, hi):
    m, h = (lo + hi) / 2, (hi - lo) / 2
    q = np.abs(p - m[:, None]) - h[:, None]
    out = np.sqrt((np.maximum(q, 0) ** 2).sum(axis=0))
    ins = np.minimum(q.max(axis=0), 0)
    return out + ins


def test_box_mesh_distance_and_inside_match_the_box():
    lo, hi = np.array([-1.0, 0.0, 2.0]), np.array([3.0, 1.5, 4.0])
    mo = MeshObstacle(*mg.box_mesh(lo, hi))
    rng = np.random.default_rng(32)
    P = rng.uniform(-3, 6, size=(3, 400))
    sd = _box_sd(P, lo, hi)
    for j in range(P.shape[1]):
        c, d2, t, psi = mo.closest(P[:, j])
        assert np.sqrt(d2) == pytest.approx(abs(sd[j]), abs=1e-12)
        inside, tc, u, _ = mo.target(P[:, j], 0.1)
        assert inside == (sd[j] < 0)
        np.testing.assert_allclose(np.linalg.norm(u), 1.0, atol=1e-14)
        # the target is eps outside the box, along u
        assert _box_sd(tc[:, None], lo, hi)[0] == pytest.approx(0.1, abs=1e-12)


def test_box_targets_in_closed_form():
    lo, hi = np.array([0.0, 0.0, 0.0]), np.array([4.0, 4.0, 4.0])
    mo = MeshObstacle(*mg.box_mesh(lo, hi))
    inside, tc, u, _ = mo.target(np.array([0.3, 2.0, 1.5]), 0.05)       # nearest face x = 0
    assert inside
    np.testing.assert_allclose(tc, [-0.05, 2.0, 1.5], atol=1e-15)
    np.testing.assert_allclose(u, [-1.0, 0.0, 0.0], atol=1e-15)
    inside, tc, u, _ = mo.target(np.array([5.0, 5.0, 2.0]), 0.05)       # outside, nearest edge
    assert not inside
    np.testing.assert_allclose(u, np.array([1.0, 1.0, 0.0]) / np.sqrt(2), atol=1e-15)
    np.testing.assert_allclose(tc, np.array([4.0, 4.0, 2.0]) + 0.05 * u, atol=1e-15)


def test_icosphere_inside_matches_the_sphere_away_from_the_facets():
    c0, r = np.array([1.0, -2.0, 0.5]), 3.0
    mo = MeshObstacle(*mg.icosphere(c0, r, 3))
    rng = np.random.default_rng(33)
    d = rng.normal(size=(3, 300))
    d /= np.linalg.norm(d, axis=0)
    rad = np.concatenate([rng.uniform(0.0, 0.97 * r, 150), rng.uniform(1.0001 * r, 2 * r, 150)])
    P = c0[:, None] + d * rad
    for j in range(P.shape[1]):
        assert mo.target(P[:, j], 0.1)[0] == (rad[j] < r)


def test_mesh_obstacle_is_checked():
    V, F = mg.box_mesh([0, 0, 0], [1, 1, 1])
    with pytest.raises(ValueError):
        MeshObstacle(V, F[:-1])                    # not closed
    with pytest.raises(ValueError):
        MeshObstacle(V, np.vstack([F, [[0, 0, 1]]]))


def test_icosphere_press_matches_the_analytic_sphere():
    """A finger pressed by an icosphere (level 4, 5,120 triangles) ends within
    the facets' depth of the same finger pressed by the analytic sphere."""
    w = pressed_finger()
    sph = w.spheres[0]
    ws = dataclasses.replace(w, planes=np.zeros((0, 6)), self_collision=False)
    wm = dataclasses.replace(ws, spheres=np.zeros((0, 4)), mesh_obstacle=mg.icosphere(sph[:3], sph[3], 4))
    ps = oracle.Problem.from_workload(ws)
    pm = oracle.Problem.from_workload(wm)
    xs, As, ss = oracle.solve(ps, w.alpha, max_iter=600, tol=1e-10, anderson=8)
    xm, Am, sm = oracle.solve(pm, w.alpha, max_iter=600, tol=1e-10, anderson=8)
    assert ss["converged"] and sm["converged"]
    rs, _ = As.listing(ps)
    rm, _ = Am.listing(pm)
    assert np.all(rs[:, 1] == SPHERE) and np.all(rm[:, 1] == MESH)
    assert rm.shape[0] > 3
    # facet depth of the level-4 icosphere: r (1 - cos(theta)), theta the
    # largest angle between a facet's centre and its corners (< 0.04 rad)
    depth = sph[3] * (1 - np.cos(0.04))
    err = np.abs(xm - xs).max()
    print("sphere contacts", rs.shape[0], "mesh contacts", rm.shape[0], "max |dx|", err, "facet depth", depth)
    assert err < 4 * depth
