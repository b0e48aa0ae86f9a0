"""Pins for the oracle's collision detection and response (Sections II-B, II-C;
Eqs. 3, 4, 5, 8)."""
import numpy as np
import pytest

from paper_2203_02054_amd import meshgen as mg
import oracle
from oracle import collision as oc
from oracle.mesh import orient
from tests.meshes import voxel_box, slit_pair


def _prob(mesh, nch=1, **kw):
    return oracle.Problem(mesh["rest_xyz"], mesh["tets"], mesh["tet_mode"], mesh["tet_chamber"],
                          mesh["fixed"], nch, oracle.Params(**kw))


def test_point_in_tet_agrees_with_barycentric_solve():
    rng = np.random.default_rng(0)
    n_in = 0
    for _ in range(2000):
        P = rng.normal(size=(3, 4))
        if orient(*(P[:, i] for i in range(4))) < 0:
            P[:, [2, 3]] = P[:, [3, 2]]
        q = P.mean(axis=1) + rng.normal(size=3) * 0.7
        A = np.vstack([P, np.ones(4)])
        lam = np.linalg.solve(A, np.append(q, 1.0))
        if np.abs(lam).min() < 1e-9:
            continue
        inside = all(orient(*[q if k == j else P[:, k] for k in range(4)]) > 0 for j in range(4))
        assert inside == bool(np.all(lam > 0))
        n_in += inside
    assert n_in > 100


def test_moller_trumbore_agrees_with_direct_solve():
    rng = np.random.default_rng(1)
    hits = 0
    for _ in range(2000):
        a = rng.normal(size=(3, 3))
        o = rng.normal(size=3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        L = 3.0
        ok, t = oc.moller_trumbore(o, d, a[:, :1], a[:, 1:2], a[:, 2:3], L)
        # o + t d = a0 + u (a1 - a0) + w (a2 - a0)
        M = np.column_stack([-d, a[:, 1] - a[:, 0], a[:, 2] - a[:, 0]])
        tt, u, w = np.linalg.solve(M, o - a[:, 0])
        margin = min(abs(u), abs(w), abs(1 - u - w), abs(tt), abs(L - tt))
        if margin < 1e-9:
            continue
        expect = u > 0 and w > 0 and u + w < 1 and 0 < tt < L
        assert bool(ok[0]) == expect
        if expect:
            assert t[0] == pytest.approx(tt, rel=1e-9)
            hits += 1
    assert hits > 50


def test_vertex_normals_point_outward_on_a_convex_box():
    mesh = voxel_box(3, 2, 2, h=1.0)
    prob = _prob(mesh)
    n, ok = oc.vertex_normals(prob, prob.X0, prob.surf_verts)
    assert ok.all()
    ctr = prob.X0.mean(axis=1, keepdims=True)
    assert np.all(np.sum(n * (prob.X0[:, prob.surf_verts] - ctr), axis=0) > 0)
    np.testing.assert_allclose(np.linalg.norm(n, axis=0), 1.0, rtol=1e-15)


def _deformed_slit(push=1.5, jitter=0.05, seed=0):
    mesh, vijk = slit_pair(h=1.0, gap=1, depth=2)
    prob = _prob(mesh, self_collision=True)
    rng = np.random.default_rng(seed)
    x = prob.X0.copy()
    right = x[0] > 2.5
    x[0, right] -= push              # the right block moves into the left one,
    x[1, right] += 0.3               # off the grid lines so that its vertices
    x[2, right] += 0.2               # fall inside tets rather than on their faces
    x += jitter * rng.normal(size=x.shape)
    return prob, x


def _loops_tet_candidates(prob, x):
    out = []
    for v in prob.query_verts:
        for e in range(prob.T):
            vs = prob.tets[:, e]
            if v in vs:
                continue
            lo, hi = x[:, vs].min(axis=1), x[:, vs].max(axis=1)
            if np.all(lo <= x[:, v]) and np.all(x[:, v] <= hi):
                out.append((int(v), e))
    return out


def test_tet_candidates_match_double_loop():
    prob, x = _deformed_slit()
    v, e, inside = oc.tet_candidates(prob, x, prob.query_verts, chunk=7)
    got = sorted(zip(v.tolist(), e.tolist()))
    assert got == list(zip(v.tolist(), e.tolist()))        # already sorted by (v, e)
    assert got == _loops_tet_candidates(prob, x)
    assert inside.sum() > 0


def test_slit_closing_detects_and_targets_the_opposite_face():
    """A block pushed 1.4 mm across a 1 mm slit: the two facing boundary layers
    interpenetrate.  Each penetrating vertex marches along its inverse normal to the
    other block's facing boundary and gets a target an offset eps beyond it
    (Section II-C)."""
    prob, x = _deformed_slit(push=1.4, jitter=0.0)
    A, info = oc.collide(prob, x)
    pen_v = prob.query_verts[info["pen_self"]]
    rest_x = prob.X0[0, pen_v]
    assert set(rest_x.tolist()) == {2.0, 3.0}
    rows, tg = A.listing(prob)
    assert sorted(rows[:, 0].tolist()) == sorted(pen_v.tolist())
    eps = prob.eps_off
    n, ok = oc.vertex_normals(prob, x, rows[:, 0])
    assert ok.all()
    for i, (r, t) in enumerate(zip(rows, tg)):
        v = r[0]
        f = prob.faces[r[2]]
        plane_x = 2.0 if prob.X0[0, v] == 3.0 else 3.0 - 1.4
        # the hit lies on the other block's facing boundary; the target is eps further
        # along the inverse normal
        hit = t + eps * n[:, i]
        assert hit[0] == pytest.approx(plane_x, abs=1e-12)
        assert np.all(np.abs(x[0, f] - plane_x) < 1e-12)
        assert np.linalg.norm(t - x[:, v]) <= prob.L_ray + eps


def test_sphere_and_plane_targets_closed_form():
    eps = 0.05
    sph = np.array([1.0, -2.0, 0.5, 3.0])
    x = np.array([2.0, -1.0, 1.0])
    c, n = oc.sphere_target(x, sph, eps)
    assert np.linalg.norm(c - sph[:3]) == pytest.approx(3.0 + eps, rel=1e-14)
    np.testing.assert_allclose(n, (x - sph[:3]) / np.linalg.norm(x - sph[:3]), rtol=1e-14)
    pl = np.array([0.0, 0.0, -1.0, 0.0, 0.0, 1.0])
    c, n = oc.plane_target(np.array([0.3, 0.4, -1.2]), pl, eps)
    np.testing.assert_allclose(c, [0.3, 0.4, -1.0 + eps], atol=1e-15)


def test_release_rule_eq8_for_plane_and_self_springs():
    """A spring is kept while |n . (x - c)| <= eps and released beyond (Eq. 8)."""
    mesh = voxel_box(1, 1, 1, h=1.0)
    pl = np.array([[0.0, 0.0, -0.5, 0.0, 0.0, 1.0]])
    prob = oracle.Problem(mesh["rest_xyz"], mesh["tets"], mesh["tet_mode"], mesh["tet_chamber"],
                          mesh["fixed"], 1, oracle.Params(obstacle_collision=True, self_collision=True),
                          None, pl)
    eps = prob.eps_off
    x = prob.X0.copy()
    x[2] -= 0.5 + 0.1                                  # the bottom face dips below the plane
    A1, _ = oc.collide(prob, x)
    bottom = prob.query_verts[prob.X0[2, prob.query_verts] == 0]
    rows, _ = A1.listing(prob)
    assert sorted(rows[:, 0].tolist()) == sorted(bottom.tolist())
    assert set(rows[:, 1].tolist()) == {oc.PLANE}
    for s_above, keep in [(1.5 * eps, True), (2.5 * eps, False)]:
        y = prob.X0.copy()
        y[2] = prob.X0[2] - 0.5 + s_above                # bottom face at s_above over the plane
        A2, _ = oc.collide(prob, y, A1)
        assert (A2.count == len(bottom)) == keep
    # a kept self spring keeps its stored target; release once it is more than eps away
    S = prob.query_verts.size
    prev = oc.Contacts.empty(S, prob.n_slots)
    prev.active[0, 0] = True
    v = prob.query_verts[0]
    prev.normal[0, 0] = [1.0, 0.0, 0.0]
    prev.target[0, 0] = prob.X0[:, v] + [0.5 * eps, 0.0, 0.0]
    A3, _ = oc.collide(prob, prob.X0, prev)
    assert A3.active[0, 0] and np.array_equal(A3.target[0, 0], prev.target[0, 0])
    prev.target[0, 0] = prob.X0[:, v] + [1.5 * eps, 0.0, 0.0]
    A4, _ = oc.collide(prob, prob.X0, prev)
    assert not A4.active[0, 0]


def test_ray_candidates_match_double_loop():
    prob, x = _deformed_slit(push=1.5, jitter=0.03, seed=2)
    A, info = oc.collide(prob, x)
    cv, cf = info["cand_tri"]
    pen = prob.query_verts[info["pen_self"]]
    n, ok = oc.vertex_normals(prob, x, pen)
    L = prob.L_ray
    expect = []
    for i, v in enumerate(pen):
        if not ok[i]:
            continue
        o, d = x[:, v], -n[:, i]
        end = o + L * d
        slo, shi = np.minimum(o, end), np.maximum(o, end)
        for f, tri in enumerate(prob.faces):
            if v in tri:
                continue
            flo, fhi = x[:, tri].min(axis=1), x[:, tri].max(axis=1)
            if np.all(flo <= shi) and np.all(slo <= fhi):
                expect.append((int(v), f))
    assert sorted(zip(cv.tolist(), cf.tolist())) == expect
    assert len(expect) > 0


def test_vertex_normals_are_area_weighted_on_an_anisotropic_voxel():
    """One voxel stretched to 1 x 2 x 3 (Kuhn split: every face diagonal starts
    at the lower corner of its face).  Each boundary triangle adds its cross
    product, twice its area along its outward normal, so the corner (0,0,0),
    met by two triangles on each of its three faces, has the normal
    -(b c, a c, a b) / |.| = -(6, 3, 2) / 7, and the corner (a,0,0), met by two
    triangles on the face x = a and one on each of the others, has
    (2 b c, -a c, -a b) / |.| = (12, -3, -2) / sqrt(157).  An unweighted sum
    of unit face normals would give (1, 1, 1) / sqrt(3) and (2, -1, -1) /
    sqrt(6) instead."""
    mesh = voxel_box(1, 1, 1, h=1.0)
    mesh["rest_xyz"] = mesh["rest_xyz"] * np.array([[1.0], [2.0], [3.0]])
    prob = _prob(mesh)
    corner0 = int(np.nonzero(np.all(prob.X0.T == [0.0, 0.0, 0.0], axis=1))[0][0])
    corner1 = int(np.nonzero(np.all(prob.X0.T == [1.0, 0.0, 0.0], axis=1))[0][0])
    n, ok = oc.vertex_normals(prob, prob.X0, np.array([corner0, corner1]))
    assert ok.all()
    exp0 = -np.array([6.0, 3.0, 2.0]) / 7.0
    exp1 = np.array([12.0, -3.0, -2.0]) / np.sqrt(157.0)
    np.testing.assert_allclose(n[:, 0], exp0, atol=1e-15)
    np.testing.assert_allclose(n[:, 1], exp1, atol=1e-15)
    # the mistake this pins: unit face normals summed without their areas
    assert np.abs(n[:, 0] + np.ones(3) / np.sqrt(3)).max() > 0.1
    assert np.abs(n[:, 1] - np.array([2.0, -1.0, -1.0]) / np.sqrt(6)).max() > 0.1


@pytest.mark.parametrize("seed", [0, 1])
def test_kdtree_broadphase_finds_the_brute_force_pairs(seed):
    """The k-d tree broadphase returns exactly the brute-force candidate pairs
    and penetration flags (deformed slit with jitter, and a pressed finger
    state with contacts), and the collision response built on it is the same."""
    prob, x = _deformed_slit(seed=seed)
    a = oc.tet_candidates(prob, x, prob.query_verts)
    b = oc.tet_candidates(prob, x, prob.query_verts, broadphase="kdtree")
    for u, w in zip(a, b):
        np.testing.assert_array_equal(u, w)
    assert a[2].any()
    from tests.meshes import pressed_finger
    w = pressed_finger()
    pf = oracle.Problem.from_workload(w)
    xs, A, _ = oracle.solve(pf, w.alpha, fixed_iters=20 + seed)
    a = oc.tet_candidates(pf, xs, pf.query_verts)
    b = oc.tet_candidates(pf, xs, pf.query_verts, broadphase="kdtree")
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)
    A1, _ = oracle.collide(pf, xs, A)
    A2, _ = oracle.collide(pf, xs, A, broadphase="kdtree")
    assert A1.same_set(A2) and np.array_equal(A1.target, A2.target) and np.array_equal(A1.prim, A2.prim)
