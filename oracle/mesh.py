"""Oracle set-up: the element model of Section II-A and the fixed system matrix.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Everything is FP64 numpy.  The quantities follow the paper's element model:

* a tet stores V_e = [v1 v2 v3 v4] (3x4; Section II-A);
* N = I_4 - 1/4 * 1 1^T removes translation (below Eq. 1).  The paper writes
  "N V", which does not conform with a 3x4 V; the centring is applied on the
  right, V N (reading 1);
* Vol(e) is the signed volume of the rest tet; every element gets the weight
  omega_e = Vol(e) / mean Vol (Eq. 9 weights, reading 6);
* the global matrix of the least-squares problem of Eq. 9 is
  A_el = sum_e omega_e S_e^T N S_e (S_e selects the tet's vertices).
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np
import scipy.sparse as sp

# Canonical orientation: a tet whose rest orient() is negative swaps its
# slots 2 and 3.  The GPU library applies the same rule so that tet-local
# orders (and therefore the exact predicates) agree.
ORIENT_SWAP = (2, 3)

# outward faces of a positively oriented tet (a,b,c,d): the face opposite slot m
FACE_SLOTS = ((1, 2, 3), (0, 3, 2), (0, 1, 3), (0, 2, 1))

BODY, CH_ISO, CH_AX_X, CH_AX_Y, CH_AX_Z = 0, 1, 2, 3, 4


@dataclass
class Params:
    """Solver constants (paper values where the paper gives them)."""

    c1: float = 0.0418            # Mooney-Rivlin, Ecoflex 00-30 (Section IV-A), MPa
    c2: float = 0.0106
    hyperelastic: bool = True     # False: R_w == 1 (as-rigid-as-possible targets)
    kappa_col: float = 1.0        # spring stiffness k_v = kappa_col * A_el[v, v]
    eps_rel: float = 0.05         # offset of the collided boundary (Section II-C), x h_ref
    ray_rel: float = 4.0          # length of the inverse-normal search, x h_ref
    self_collision: bool = False
    obstacle_collision: bool = False
    tol: float = 1e-6             # outer residual, relative to the bounding-box diagonal
    max_iter: int = 1000
    fixed_iters: int = 0          # >0: run exactly this many iterations

    def with_(self, **kw) -> "Params":
        return replace(self, **kw)


def orient(p0, p1, p2, p3):
    """Six times the signed volume det[p1-p0, p2-p0, p3-p0].

    Arrays have the coordinate on axis 0.  Evaluated in the fixed order
    written below (no fused multiply-add: numpy never fuses), so the GPU's
    predicate, written in the same order with contraction off, returns the
    same bits from the same inputs.
    """
    ax, ay, az = p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]
    bx, by, bz = p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]
    cx, cy, cz = p3[0] - p0[0], p3[1] - p0[1], p3[2] - p0[2]
    return ax * (by * cz - bz * cy) + ay * (bz * cx - bx * cz) + az * (bx * cy - by * cx)


def centring() -> np.ndarray:
    """N = I_4 - 1/4 * ones (below Eq. 1)."""
    return np.eye(4) - 0.25 * np.ones((4, 4))


class Problem:
    """Rest-state data for one mesh (set-up step, done once per mesh)."""

    def __init__(self, rest_xyz, tets, tet_mode, tet_chamber, fixed, n_chambers,
                 params: Params | None = None, spheres=None, planes=None, mesh_obstacle=None):
        self.params = params or Params()
        X = np.ascontiguousarray(rest_xyz, dtype=np.float64)
        tets = np.array(tets, dtype=np.int64, copy=True)
        n = X.shape[1]
        T = tets.shape[1]
        if X.shape[0] != 3 or tets.shape[0] != 4:
            raise ValueError("rest_xyz must be [3,n] and tets [4,T]")
        if T == 0 or n == 0:
            raise ValueError("empty mesh")
        if tets.min() < 0 or tets.max() >= n:
            raise ValueError("tet index out of range")
        if not np.all(np.isfinite(X)):
            raise ValueError("non-finite rest position")
        self.n, self.T = n, T
        self.X0 = X
        self.mode = np.asarray(tet_mode, dtype=np.int64)
        self.chamber = np.asarray(tet_chamber, dtype=np.int64)
        self.fixed = np.asarray(fixed).astype(bool)
        self.n_chambers = int(n_chambers)
        if np.any((self.mode != BODY) & ((self.chamber < 0) | (self.chamber >= self.n_chambers))):
            raise ValueError("chamber element without a valid chamber id")

        # h_ref: mean rest length of the unique tet edges
        e = np.concatenate([np.sort(tets[[a, b]], axis=0) for a in range(4) for b in range(a + 1, 4)], axis=1)
        e = np.unique(e[0] * n + e[1])
        ei, ej = e // n, e % n
        d = X[:, ei] - X[:, ej]
        lens = np.sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])
        # summed in ascending (i, j) edge order, one term at a time, so that the
        # offsets eps and L_ray derived from h_ref are reproducible bit for bit
        acc = 0.0
        for v in lens.tolist():
            acc += v
        self.h_ref = acc / lens.size

        # orientation: positive rest volume; swap slots 2 and 3 otherwise
        v6 = orient(X[:, tets[0]], X[:, tets[1]], X[:, tets[2]], X[:, tets[3]])
        if np.any(np.abs(v6) / 6.0 <= 1e-12 * self.h_ref ** 3):
            raise ValueError("degenerate rest tet")
        neg = v6 < 0
        a, b = ORIENT_SWAP
        tets[a, neg], tets[b, neg] = tets[b, neg].copy(), tets[a, neg].copy()
        self.tets = tets

        Xe = X[:, tets]                                  # [3, 4, T]
        self.Xe = np.moveaxis(Xe, 2, 0)                  # [T, 3, 4]
        self.P = self.Xe @ centring()                    # rest shape X_e N
        self.Dm = self.Xe[:, :, 1:] - self.Xe[:, :, :1]  # [T, 3, 3]
        self.Dm_inv = np.linalg.inv(self.Dm)
        self.vol = np.linalg.det(self.Dm) / 6.0
        self.omega = self.vol / self.vol.mean()

        lo, hi = X.min(axis=1), X.max(axis=1)
        self.diag = float(np.linalg.norm(hi - lo))
        self.eps_off = self.params.eps_rel * self.h_ref
        self.L_ray = self.params.ray_rel * self.h_ref

        # A_el = sum_e omega_e S_e^T N S_e
        Nm = centring()
        rows = np.repeat(tets, 4, axis=0).reshape(4, 4, T)          # rows[a, b] = tets[a]
        cols = np.tile(tets, (4, 1)).reshape(4, 4, T)               # cols[a, b] = tets[b]
        vals = Nm[:, :, None] * self.omega[None, None, :]
        self.A_el = sp.csr_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=(n, n))
        self.A_el.sum_duplicates()
        self.A_diag = self.A_el.diagonal().copy()
        self.k_spring = self.params.kappa_col * self.A_diag

        # boundary faces (belonging to exactly one tet), outward, in (tet, slot) order
        fv = np.stack([tets[list(s)] for s in FACE_SLOTS], axis=0)   # [4 slots, 3, T]
        fv = np.transpose(fv, (2, 0, 1)).reshape(4 * T, 3)           # (e, m) order
        key = np.sort(fv, axis=1)
        kk = (key[:, 0] * n + key[:, 1]) * n + key[:, 2]
        _, inv, cnt = np.unique(kk, return_inverse=True, return_counts=True)
        on_surf = cnt[inv] == 1
        self.faces = fv[on_surf]                                     # [F, 3]
        self.surf_verts = np.unique(self.faces)
        self.query_verts = self.surf_verts[~self.fixed[self.surf_verts]]

        sph = np.zeros((0, 4)) if spheres is None else np.asarray(spheres, dtype=np.float64).reshape(-1, 4)
        pln = np.zeros((0, 6)) if planes is None else np.asarray(planes, dtype=np.float64).reshape(-1, 6)
        if pln.shape[0]:
            nrm = np.sqrt((pln[:, 3] * pln[:, 3] + pln[:, 4] * pln[:, 4]) + pln[:, 5] * pln[:, 5])
            if np.any(nrm == 0):
                raise ValueError("plane with zero normal")
            pln = pln.copy()
            pln[:, 3:] = pln[:, 3:] / nrm[:, None]
        if sph.shape[0] and np.any(sph[:, 3] <= 0):
            raise ValueError("sphere with non-positive radius")
        self.spheres, self.planes = sph, pln
        # a closed triangle-mesh obstacle ((verts [3, m], tris [k, 3]) or None)
        self.mesh_obstacle = None
        if mesh_obstacle is not None:
            from .obstacle import MeshObstacle
            self.mesh_obstacle = MeshObstacle(*mesh_obstacle)

        self.free = ~self.fixed

    @classmethod
    def from_workload(cls, wl, params: Params | None = None, **kw):
        p = params or Params(c1=wl.material[0], c2=wl.material[1],
                             self_collision=wl.self_collision,
                             obstacle_collision=wl.obstacle_collision,
                             fixed_iters=wl.fixed_iters)
        if kw:
            p = p.with_(**kw)
        return cls(wl.rest_xyz, wl.tets, wl.tet_mode, wl.tet_chamber, wl.fixed,
                   wl.n_chambers, p, wl.spheres, wl.planes, getattr(wl, "mesh_obstacle", None))

    @property
    def n_slots(self) -> int:
        """Contact slots per query vertex: self, then each sphere, then each
        plane, then one for the triangle-mesh obstacle if there is one."""
        return 1 + self.spheres.shape[0] + self.planes.shape[0] + (self.mesh_obstacle is not None)
