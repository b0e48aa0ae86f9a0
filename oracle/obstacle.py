"""Oracle: triangle-mesh obstacles (Section II-B, obstacle term of Eq. 4;
Section II-C, the target on the collided boundary).

TEST INFRASTRUCTURE ONLY (see the package docstring).

An obstacle may be a closed, outward-oriented triangle mesh instead of an
analytic sphere or plane.  A query vertex p is tested against it through its
closest point c on the mesh (brute force over every triangle, which is the
definition; any tree must reproduce it):

* closest point on one triangle: the Voronoi-region walk of Ericson,
  Real-Time Collision Detection (2005), Section 5.1.5, written out below in
  a fixed order of operations (no fused multiply-add);
* over the mesh: the smallest squared distance |p - c|^2 wins, ties to the
  lowest triangle id;
* inside: (p - c) . psi < 0, with psi the angle-weighted pseudonormal of the
  feature (face, edge or vertex) that c lies on (Baerentzen and Aanaes, 2005:
  face normal; for an edge the sum of its two faces' unit normals; for a
  vertex the sum of its faces' unit normals weighted by their angles there).
  This sign is exact for a closed 2-manifold; p on the surface is outside.

Response (reading of the obstacle case of Section II-C): the outward unit
direction u from the surface towards the outside at p is (p - c)/|p - c|
when p is outside, (c - p)/|p - c| when inside, psi when p = c; the target
is c + eps u and the contact normal u, recomputed at every check as for the
analytic obstacles (so the release rule of Eq. 8 drops a kept contact once
p is more than 2 eps outside, as for a plane).
"""
from __future__ import annotations

import numpy as np

FACE, EDGE, VERTEX = 0, 1, 2


def _dot(a, b):
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]


def _cross(a, b):
    return np.stack([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]])


def closest_on_triangles(p, a, b, c):
    """Closest points of p [3] on the triangles (a, b, c) [3, K] and the
    feature each lies on: (point [3, K], kind [K] FACE/EDGE/VERTEX, local
    index [K]: vertex 0/1/2 of (a, b, c), or edge 0 = ab, 1 = ac, 2 = bc)."""
    p = np.asarray(p, dtype=np.float64).reshape(3, 1)
    K = a.shape[1]
    ab, ac, ap = b - a, c - a, p - a
    d1, d2 = _dot(ab, ap), _dot(ac, ap)
    bp = p - b
    d3, d4 = _dot(ab, bp), _dot(ac, bp)
    cp = p - c
    d5, d6 = _dot(ab, cp), _dot(ac, cp)
    vc = d1 * d4 - d3 * d2
    vb = d5 * d2 - d1 * d6
    va = d3 * d6 - d5 * d4
    out = np.empty((3, K))
    kind = np.full(K, FACE, np.int64)
    loc = np.zeros(K, np.int64)
    done = np.zeros(K, bool)

    def put(mask, pt, k, i):
        m = mask & ~done
        out[:, m] = pt[:, m] if pt.ndim == 2 else pt
        kind[m] = k
        loc[m] = i
        done[m] = True

    with np.errstate(divide="ignore", invalid="ignore"):
        put((d1 <= 0) & (d2 <= 0), a, VERTEX, 0)
        put((d3 >= 0) & (d4 <= d3), b, VERTEX, 1)
        t = d1 / (d1 - d3)
        put((vc <= 0) & (d1 >= 0) & (d3 <= 0), a + t * ab, EDGE, 0)
        put((d6 >= 0) & (d5 <= d6), c, VERTEX, 2)
        t = d2 / (d2 - d6)
        put((vb <= 0) & (d2 >= 0) & (d6 <= 0), a + t * ac, EDGE, 1)
        e43, e56 = d4 - d3, d5 - d6
        t = e43 / (e43 + e56)
        put((va <= 0) & (e43 >= 0) & (e56 >= 0), b + t * (c - b), EDGE, 2)
        den = 1.0 / ((va + vb) + vc)
        v, w = vb * den, vc * den
        put(np.ones(K, bool), a + ab * v + ac * w, FACE, 0)
    return out, kind, loc


class MeshObstacle:
    """A closed, outward-oriented triangle mesh: verts [3, m], tris [k, 3]."""

    def __init__(self, verts, tris):
        V = np.ascontiguousarray(verts, dtype=np.float64)
        F = np.ascontiguousarray(tris, dtype=np.int64)
        if V.ndim != 2 or V.shape[0] != 3 or F.ndim != 2 or F.shape[1] != 3 or F.shape[0] == 0:
            raise ValueError("mesh obstacle: verts [3, m] and tris [k, 3]")
        if F.min() < 0 or F.max() >= V.shape[1]:
            raise ValueError("mesh obstacle: triangle index out of range")
        self.V, self.F = V, F
        a, b, c = V[:, F[:, 0]], V[:, F[:, 1]], V[:, F[:, 2]]
        n = _cross(b - a, c - a)
        ln = np.sqrt(_dot(n, n))
        if np.any(ln == 0):
            raise ValueError("mesh obstacle: degenerate triangle")
        self.fn = n / ln                                          # [3, k] unit face normals
        # edges: each undirected edge must be shared by exactly two faces
        k = F.shape[0]
        e = np.sort(np.stack([F[:, [0, 1]], F[:, [0, 2]], F[:, [1, 2]]], axis=1), axis=2)  # [k, 3, 2]
        key = e[:, :, 0] * V.shape[1] + e[:, :, 1]
        uniq, inv, cnt = np.unique(key.ravel(), return_inverse=True, return_counts=True)
        if np.any(cnt != 2):
            raise ValueError("mesh obstacle: not a closed 2-manifold (an edge is not shared by two faces)")
        en = np.zeros((3, uniq.size))
        np.add.at(en.T, inv, np.repeat(self.fn.T, 3, axis=0))
        self.edge_id = inv.reshape(k, 3)                         # local edge (ab, ac, bc) -> global
        self.en = en / np.sqrt(_dot(en, en))
        # vertices: angle-weighted sum of the incident faces' normals
        vn = np.zeros_like(V)
        P = [a, b, c]
        for i in range(3):
            u, w = P[(i + 1) % 3] - P[i], P[(i + 2) % 3] - P[i]
            cosang = _dot(u, w) / np.sqrt(_dot(u, u) * _dot(w, w))
            ang = np.arccos(np.clip(cosang, -1.0, 1.0))
            np.add.at(vn.T, F[:, i], (self.fn * ang).T)
        self.vn = vn / np.sqrt(_dot(vn, vn))
        self.lo, self.hi = V.min(axis=1), V.max(axis=1)

    @property
    def n_tris(self) -> int:
        return self.F.shape[0]

    def closest(self, p):
        """(c [3], squared distance, triangle id, pseudonormal psi [3])."""
        a, b, c = self.V[:, self.F[:, 0]], self.V[:, self.F[:, 1]], self.V[:, self.F[:, 2]]
        q, kind, loc = closest_on_triangles(p, a, b, c)
        p = np.asarray(p, dtype=np.float64)
        dx, dy, dz = p[0] - q[0], p[1] - q[1], p[2] - q[2]
        d2 = (dx * dx + dy * dy) + dz * dz
        t = int(np.argmin(d2))                   # first of the smallest: lowest id on ties
        if kind[t] == FACE:
            psi = self.fn[:, t]
        elif kind[t] == EDGE:
            psi = self.en[:, self.edge_id[t, loc[t]]]
        else:
            psi = self.vn[:, self.F[t, loc[t]]]
        return q[:, t], float(d2[t]), t, psi

    def target(self, p, eps):
        """(inside, target [3], outward normal u [3], triangle id) at p."""
        p = np.asarray(p, dtype=np.float64)
        c, d2, t, psi = self.closest(p)
        g = p - c
        inside = _dot(g, psi) < 0.0
        if d2 > 0.0:
            dist = np.sqrt(d2)
            u = g / dist if not inside else -g / dist
        else:
            u = psi.copy()
        tc = np.array([c[0] + eps * u[0], c[1] + eps * u[1], c[2] + eps * u[2]])
        return bool(inside), tc, u, t
