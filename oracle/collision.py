"""Oracle collision detection and response (Sections II-B, II-C, III-A.3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Brute force over all pairs *is* the definition of the candidate sets; any
broadphase (the paper's AABB tree, the GPU's spatial hash) must reproduce them
exactly.  Every predicate is evaluated in FP64 in the order written here.

Detection (Eq. 3, Eq. 4).  The query vertices are the non-fixed boundary
vertices of the tet mesh (reading 9).  The tet candidates of a query vertex v
are C_tet = {(v, e): v not a vertex of e, lo_e <= x_v <= hi_e on every axis},
with [lo_e, hi_e] the min/max box of e's four vertices.  v penetrates e when
all four sub-volumes obtained by replacing one vertex of e with v are
strictly positive (ties count as outside).  Obstacles: inside a sphere when
|x - c|^2 < r^2, below a plane when n . (x - p) < 0.

A closed triangle-mesh obstacle (``oracle.obstacle``) is tested through the
closest point on it: inside when the offset from that point points against
the feature's pseudonormal.

Response (Eq. 5, Section II-C).  A penetrating vertex gets a virtual spring to
a target v_c.  Self collision: march from x_v along the inverse vertex normal
-n(v) (area-weighted sum of the incident boundary-face normals) to the first
boundary triangle not incident to v, within L_ray = 4 h_ref (Moller-Trumbore
test; ties to the lowest face id), and put the target an offset eps past the
hit (reading 10).  Obstacles: the closest point on the offset surface.

Active set with release rule (Eq. 8).  For each query vertex (ascending) and
each contact slot (self, then spheres, then planes, then the mesh obstacle): a penetrating vertex gets
a fresh spring; otherwise a spring it already had is kept unless
|n_c . (x_v - c)| > eps (n_c = the stored contact normal, reading 11; obstacle
springs recompute c and n_c first, kept self springs keep their stored target,
reading 12).  A penetrating vertex whose ray finds no triangle adds no spring
(counted as a ray miss) but keeps a previous self spring.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .mesh import orient

SELF, SPHERE, PLANE, MESH = 0, 1, 2, 3


@dataclass
class Contacts:
    """Dense active set: one row per query vertex, one column per slot."""

    active: np.ndarray            # [S, n_slots] bool
    target: np.ndarray            # [S, n_slots, 3] float64
    normal: np.ndarray            # [S, n_slots, 3] float64
    prim: np.ndarray              # [S, n_slots] int64 (hit face / obstacle index)

    @classmethod
    def empty(cls, S: int, n_slots: int) -> "Contacts":
        return cls(np.zeros((S, n_slots), bool), np.zeros((S, n_slots, 3)),
                   np.zeros((S, n_slots, 3)), np.full((S, n_slots), -1, np.int64))

    def copy(self) -> "Contacts":
        return Contacts(self.active.copy(), self.target.copy(), self.normal.copy(), self.prim.copy())

    def listing(self, prob):
        """Active contacts as sorted (v, type, prim) rows plus targets [k,3]."""
        s, slot = np.nonzero(self.active)              # row-major = (v ascending, slot ascending)
        v = prob.query_verts[s]
        ns = prob.spheres.shape[0]
        npl = prob.planes.shape[0]
        typ = np.where(slot == 0, SELF, np.where(slot <= ns, SPHERE, np.where(slot <= ns + npl, PLANE, MESH)))
        prim = self.prim[s, slot]
        return np.stack([v, typ, prim], axis=1).astype(np.int64), self.target[s, slot]

    def same_set(self, other: "Contacts") -> bool:
        return bool(np.array_equal(self.active, other.active))

    @property
    def count(self) -> int:
        return int(self.active.sum())


def _cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def _dot(a, b):
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]


def _incidence(prob):
    """Boundary faces incident to each boundary vertex, ascending face id."""
    inc = getattr(prob, "_vf_inc", None)
    if inc is None:
        F = prob.faces.shape[0]
        v = prob.faces.reshape(-1)
        f = np.repeat(np.arange(F), 3)
        order = np.lexsort((f, v))
        v, f = v[order], f[order]
        start = np.searchsorted(v, np.arange(prob.n + 1))
        inc = (start, f)
        prob._vf_inc = inc
    return inc


def vertex_normals(prob, x: np.ndarray, verts: np.ndarray):
    """Unit area-weighted normals at the given boundary vertices.

    The raw normal is the sum, in ascending face id, of (x_j - x_i) x (x_k - x_i)
    over the vertex's boundary faces (i, j, k); it is divided by its length.
    Returns (n [3, len(verts)], ok [len(verts)] where the length is non-zero).
    """
    start, finc = _incidence(prob)
    fa = prob.faces
    p0, p1, p2 = x[:, fa[:, 0]], x[:, fa[:, 1]], x[:, fa[:, 2]]
    e1 = (p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2])
    e2 = (p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2])
    cr = np.stack(_cross(e1, e2))                      # [3, F]
    verts = np.asarray(verts, dtype=np.int64)
    deg = start[verts + 1] - start[verts]
    acc = np.zeros((3, verts.size))
    for j in range(int(deg.max()) if verts.size else 0):
        sel = deg > j
        acc[:, sel] = acc[:, sel] + cr[:, finc[start[verts[sel]] + j]]
    ln = np.sqrt((acc[0] * acc[0] + acc[1] * acc[1]) + acc[2] * acc[2])
    ok = ln > 0
    with np.errstate(invalid="ignore", divide="ignore"):
        n = acc / ln
    return n, ok


def _box_pairs_kdtree(x, lo, hi, qverts):
    """(query index, tet) pairs whose inclusive box test passes, found through
    a k-d tree of the query vertices: each tet's box lies inside the ball
    around its centre with the half diagonal as radius (widened by a relative
    1e-9 for rounding), so the ball query returns every vertex of the box and
    the box test below, the same comparisons as the brute force, decides."""
    from scipy.spatial import cKDTree
    ctr = 0.5 * (lo + hi)
    rad = 0.5 * np.sqrt(((hi - lo) ** 2).sum(axis=0))
    rad = rad * (1.0 + 1e-9) + 1e-12 * (np.abs(ctr).max() + 1.0)
    tree = cKDTree(np.ascontiguousarray(x[:, qverts].T))
    lists = tree.query_ball_point(np.ascontiguousarray(ctr.T), rad, workers=-1)
    lens = np.fromiter((len(l) for l in lists), dtype=np.int64, count=len(lists))
    ei = np.repeat(np.arange(lo.shape[1], dtype=np.int64), lens)
    si = np.fromiter((i for l in lists for i in l), dtype=np.int64, count=int(lens.sum()))
    p = x[:, qverts[si]]
    m = np.ones(si.size, dtype=bool)
    for ax in range(3):
        m &= p[ax] >= lo[ax, ei]
        m &= p[ax] <= hi[ax, ei]
    si, ei = si[m], ei[m]
    order = np.lexsort((ei, si))
    return si[order], ei[order]


def tet_candidates(prob, x: np.ndarray, qverts: np.ndarray, chunk: int = 0, broadphase: str = "brute"):
    """C_tet as (v, e) arrays sorted by (v, e), and the penetration flag per pair.

    broadphase "brute" tests every (vertex, tet) pair (the definition);
    "kdtree" finds the same pairs through a k-d tree of the query vertices
    (for full-size meshes; checked equal to the brute force in the tests)."""
    tets = prob.tets
    T = tets.shape[1]
    xe = x[:, tets]                                     # [3, 4, T]
    lo = xe.min(axis=1)
    hi = xe.max(axis=1)
    if broadphase == "kdtree":
        qv = np.asarray(qverts, dtype=np.int64)
        si, ei = _box_pairs_kdtree(x, lo, hi, qv)
        v = qv[si]
        inc = (tets[:, ei] == v[None, :]).any(axis=0)
        v, e = v[~inc], ei[~inc]
        a, b, c, d = (x[:, tets[k, e]] for k in range(4))
        pv = x[:, v]
        inside = ((orient(pv, b, c, d) > 0) & (orient(a, pv, c, d) > 0)
                  & (orient(a, b, pv, d) > 0) & (orient(a, b, c, pv) > 0))
        return v.astype(np.int64), e.astype(np.int64), inside
    if broadphase != "brute":
        raise ValueError("broadphase must be 'brute' or 'kdtree'")
    chunk = chunk or max(1, min(4096, int(2e7 // max(T, 1))))
    vs, es = [], []
    for s0 in range(0, qverts.size, chunk):
        q = qverts[s0:s0 + chunk]
        p = x[:, q]
        m = np.ones((q.size, T), dtype=bool)
        for ax in range(3):
            m &= p[ax][:, None] >= lo[ax][None, :]
            m &= p[ax][:, None] <= hi[ax][None, :]
        vi, ei = np.nonzero(m)
        v = q[vi]
        inc = (tets[:, ei] == v[None, :]).any(axis=0)
        vs.append(v[~inc])
        es.append(ei[~inc])
    v = np.concatenate(vs) if vs else np.zeros(0, np.int64)
    e = np.concatenate(es) if es else np.zeros(0, np.int64)
    a, b, c, d = (x[:, tets[k, e]] for k in range(4))
    pv = x[:, v]
    inside = ((orient(pv, b, c, d) > 0) & (orient(a, pv, c, d) > 0)
              & (orient(a, b, pv, d) > 0) & (orient(a, b, c, pv) > 0))
    return v.astype(np.int64), e.astype(np.int64), inside


def moller_trumbore(o, d, a0, a1, a2, L):
    """Segment o + t d, 0 < t <= L, against triangles (a0, a1, a2) [3, k].

    Moller & Trumbore (1997): e1 = a1 - a0, e2 = a2 - a0, pv = d x e2,
    det = e1 . pv (det == 0: parallel, no hit), tv = o - a0,
    u = (tv . pv) / det, qv = tv x e1, w = (d . qv) / det, t = (e2 . qv) / det;
    a hit needs u >= 0, w >= 0, u + w <= 1 and 0 < t <= L.
    Returns (hit [k] bool, t [k]).
    """
    k = a0.shape[1]
    e1 = (a1[0] - a0[0], a1[1] - a0[1], a1[2] - a0[2])
    e2 = (a2[0] - a0[0], a2[1] - a0[1], a2[2] - a0[2])
    dd = (np.full(k, d[0]), np.full(k, d[1]), np.full(k, d[2]))
    pvec = _cross(dd, e2)
    det = _dot(e1, pvec)
    tv = (o[0] - a0[0], o[1] - a0[1], o[2] - a0[2])
    nz = det != 0
    with np.errstate(invalid="ignore", divide="ignore"):
        u = _dot(tv, pvec) / det
        qv = _cross(tv, e1)
        w = _dot(dd, qv) / det
        t = _dot(e2, qv) / det
    ok = nz & (u >= 0) & (w >= 0) & (u + w <= 1) & (t > 0) & (t <= L)
    return ok, t


def ray_cast(prob, x: np.ndarray, verts: np.ndarray, normals: np.ndarray):
    """First hit of the segment [x_v, x_v - L_ray n_v] on non-incident boundary faces.

    Returns (hit [k] bool, face [k], t [k], candidate pairs (v, f) sorted).
    Candidate faces: not incident to v and with a box overlapping the
    segment's box (inclusive bounds); each is tested by ``moller_trumbore``.
    """
    L = prob.L_ray
    fa = prob.faces
    F = fa.shape[0]
    p0, p1, p2 = x[:, fa[:, 0]], x[:, fa[:, 1]], x[:, fa[:, 2]]
    flo = np.minimum(np.minimum(p0, p1), p2)
    fhi = np.maximum(np.maximum(p0, p1), p2)
    k = verts.size
    hit = np.zeros(k, bool)
    best_f = np.full(k, -1, np.int64)
    best_t = np.full(k, np.inf)
    cv, cf = [], []
    for i in range(k):
        v = verts[i]
        o = x[:, v]
        d = -normals[:, i]
        end = np.array([o[0] + L * d[0], o[1] + L * d[1], o[2] + L * d[2]])
        slo, shi = np.minimum(o, end), np.maximum(o, end)
        m = np.ones(F, bool)
        for ax in range(3):
            m &= (flo[ax] <= shi[ax]) & (slo[ax] <= fhi[ax])
        m &= ~(fa == v).any(axis=1)
        f = np.nonzero(m)[0]
        cv.append(np.full(f.size, v, np.int64))
        cf.append(f)
        if f.size == 0:
            continue
        ok, t = moller_trumbore(o, d, p0[:, f], p1[:, f], p2[:, f], L)
        if ok.any():
            tt = np.where(ok, t, np.inf)
            j = int(np.argmin(tt))                     # first minimum = lowest face id
            hit[i], best_f[i], best_t[i] = True, f[j], tt[j]
    cand = (np.concatenate(cv) if cv else np.zeros(0, np.int64),
            np.concatenate(cf) if cf else np.zeros(0, np.int64))
    return hit, best_f, best_t, cand


def face_normal(prob, x, f):
    fa = prob.faces[f]
    p0, p1, p2 = x[:, fa[0]], x[:, fa[1]], x[:, fa[2]]
    e1 = (p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2])
    e2 = (p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2])
    c = np.array(_cross(e1, e2))
    ln = np.sqrt((c[0] * c[0] + c[1] * c[1]) + c[2] * c[2])
    return c / ln


def sphere_target(x, sph, eps):
    """Closest point on the sphere offset by eps, and the outward normal."""
    dx, dy, dz = x[0] - sph[0], x[1] - sph[1], x[2] - sph[2]
    q = (dx * dx + dy * dy) + dz * dz
    dist = np.sqrt(q)
    if dist > 0:
        n = np.array([dx / dist, dy / dist, dz / dist])
    else:
        n = np.array([0.0, 0.0, 1.0])
    rr = sph[3] + eps
    c = np.array([sph[0] + rr * n[0], sph[1] + rr * n[1], sph[2] + rr * n[2]])
    return c, n


def plane_target(x, pl, eps):
    s = (pl[3] * (x[0] - pl[0]) + pl[4] * (x[1] - pl[1])) + pl[5] * (x[2] - pl[2])
    se = s - eps
    n = pl[3:6].copy()
    c = np.array([x[0] - se * n[0], x[1] - se * n[1], x[2] - se * n[2]])
    return c, n


def _released(x, c, n, eps) -> bool:
    g = (n[0] * (x[0] - c[0]) + n[1] * (x[1] - c[1])) + n[2] * (x[2] - c[2])
    return abs(g) > eps


def collide(prob, x: np.ndarray, prev: Contacts | None = None, want_candidates: bool = False,
            broadphase: str = "brute"):
    """Active set A_k at positions x given A_{k-1} = prev (Algorithm 1, CollisionCheck).
    ``broadphase`` is passed to ``tet_candidates``.

    Returns (Contacts, info) with info = dict(pen_self, self_fresh, ray_miss,
    cand_tet, cand_tri); self_fresh marks the self contacts given a new target
    at x (the others keep a stored one).
    """
    p = prob.params
    qv = prob.query_verts
    S, ns_, npl = qv.size, prob.spheres.shape[0], prob.planes.shape[0]
    out = Contacts.empty(S, prob.n_slots)
    if prev is None:
        prev = Contacts.empty(S, prob.n_slots)
    eps = prob.eps_off
    x = np.asarray(x, dtype=np.float64)
    info = dict(ray_miss=0, pen_self=np.zeros(S, bool), self_fresh=np.zeros(S, bool), cand_tet=None,
                cand_tri=None)

    if p.self_collision:
        v, e, inside = tet_candidates(prob, x, qv, broadphase=broadphase)
        pen_v = np.unique(v[inside])
        pen = np.isin(qv, pen_v)
        info["pen_self"] = pen
        info["cand_tet"] = (v, e)
        sidx = np.nonzero(pen)[0]
        nrm, ok = vertex_normals(prob, x, qv[sidx])
        ray_idx = sidx[ok]
        hit, bf, bt, cand = ray_cast(prob, x, qv[ray_idx], nrm[:, ok])
        info["cand_tri"] = cand
        fresh = {}
        for j, s in enumerate(ray_idx):
            if hit[j]:
                d = -nrm[:, ok][:, j]
                o = x[:, qv[s]]
                te = bt[j] + eps
                c = np.array([o[0] + te * d[0], o[1] + te * d[1], o[2] + te * d[2]])
                fresh[s] = (c, face_normal(prob, x, bf[j]), bf[j])
        info["ray_miss"] = int(pen.sum() - len(fresh))
        for s in range(S):
            if pen[s] and s in fresh:
                c, n, f = fresh[s]
                out.active[s, 0] = True
                out.target[s, 0], out.normal[s, 0], out.prim[s, 0] = c, n, f
                info["self_fresh"][s] = True
            elif prev.active[s, 0]:
                keep = True if pen[s] else not _released(x[:, qv[s]], prev.target[s, 0],
                                                         prev.normal[s, 0], eps)
                if keep:
                    out.active[s, 0] = True
                    out.target[s, 0], out.normal[s, 0] = prev.target[s, 0], prev.normal[s, 0]
                    out.prim[s, 0] = prev.prim[s, 0]

    mo = prob.mesh_obstacle
    if p.obstacle_collision and mo is not None:
        # the triangle-mesh obstacle: candidates are the vertices inside its
        # box (a vertex outside the box is outside the mesh) and those holding
        # a contact with it
        slot = 1 + ns_ + npl
        xs = x[:, qv]
        inbox = np.all((xs >= mo.lo[:, None]) & (xs <= mo.hi[:, None]), axis=0)
        for s in np.nonzero(inbox | prev.active[:, slot])[0]:
            inside, c, n, t = mo.target(xs[:, s], eps)
            if inside or (prev.active[s, slot] and not _released(xs[:, s], c, n, eps)):
                out.active[s, slot] = True
                out.target[s, slot], out.normal[s, slot], out.prim[s, slot] = c, n, t
    if p.obstacle_collision and (ns_ + npl) > 0:
        xs = x[:, qv]
        for j in range(ns_):
            sph = prob.spheres[j]
            dx, dy, dz = xs[0] - sph[0], xs[1] - sph[1], xs[2] - sph[2]
            q = (dx * dx + dy * dy) + dz * dz
            inside = q < sph[3] * sph[3]
            slot = 1 + j
            for s in np.nonzero(inside | prev.active[:, slot])[0]:
                c, n = sphere_target(xs[:, s], sph, eps)
                if inside[s] or not _released(xs[:, s], c, n, eps):
                    out.active[s, slot] = True
                    out.target[s, slot], out.normal[s, slot], out.prim[s, slot] = c, n, j
        for j in range(npl):
            pl = prob.planes[j]
            sd = (pl[3] * (xs[0] - pl[0]) + pl[4] * (xs[1] - pl[1])) + pl[5] * (xs[2] - pl[2])
            inside = sd < 0
            slot = 1 + ns_ + j
            for s in np.nonzero(inside | prev.active[:, slot])[0]:
                c, n = plane_target(xs[:, s], pl, eps)
                if inside[s] or not _released(xs[:, s], c, n, eps):
                    out.active[s, slot] = True
                    out.target[s, slot], out.normal[s, slot], out.prim[s, slot] = c, n, j
    return out, info
