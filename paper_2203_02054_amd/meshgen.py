"""Seeded synthetic workloads: voxel Kuhn tet meshes of pneumatic soft robots.

The paper's own robot geometries (a twisting robot, a soft finger, a membrane
rig; Section IV and Table I) are not public inputs, so every workload here is
a deterministic synthetic stand-in with the same structure: a tetrahedral
mesh split into chamber elements (M_c) and body elements (M_b) (Section II-A),
a fixed root, per-chamber volume ratios alpha (Eq. 2) and analytic obstacles
(Eq. 4).

This module only *generates inputs*.  It holds none of the method's
arithmetic (no orientation fix, no surface extraction, no rest-shape data):
both the CPU oracle and the GPU library derive those themselves from the raw
arrays produced here.

Mesh recipe
-----------
* Each solid voxel splits into the 6 Kuhn tets {000, e_p1, e_p1+e_p2, 111},
  one per permutation p of the axes (itertools order).  The same split in
  every voxel makes the mesh conforming.  Raw tets keep the orientation the
  split gives them (half are negatively oriented on purpose).
* Grid vertices are numbered lexicographically (i*(ny+1)+j)*(nz+1)+k, unused
  ones dropped and the rest compacted in that order; tets follow voxel order.
* Units are millimetres; random numbers come from numpy's PCG64
  (``numpy.random.default_rng(seed)``).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

# Element classes (chamber elements carry how their target volume is reached).
BODY, CH_ISO, CH_AX_X, CH_AX_Y, CH_AX_Z = 0, 1, 2, 3, 4

# Mooney-Rivlin constants quoted in Section IV (MPa).
ECOFLEX_0030 = (0.0418, 0.0106)
DRAGON_SKIN_20 = (0.119, 0.023)

_PERMS = list(itertools.permutations(range(3)))


@dataclass
class Workload:
    """Raw mesh + actuation + obstacles for one robot (host arrays, FP64/int)."""

    name: str
    rest_xyz: np.ndarray          # [3, n] float64
    tets: np.ndarray              # [4, T] int32, raw orientation
    tet_mode: np.ndarray          # [T] uint8  (BODY / CH_*)
    tet_chamber: np.ndarray       # [T] int16  (-1 for body)
    fixed: np.ndarray             # [n] uint8  (1 = held at rest position)
    alpha: np.ndarray             # [n_chambers] float64 volume ratios
    spheres: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))  # cx,cy,cz,r
    planes: np.ndarray = field(default_factory=lambda: np.zeros((0, 6)))   # px,py,pz,nx,ny,nz
    # triangle-mesh obstacle: (verts [3, m], tris [k, 3]) of a closed,
    # outward-oriented mesh, or None
    mesh_obstacle: tuple | None = None
    self_collision: bool = False
    obstacle_collision: bool = False
    precision: int = 4
    fixed_iters: int = 0
    material: tuple = ECOFLEX_0030
    info: dict = field(default_factory=dict)
    # solver settings the workload is run with (passed to the library's
    # parameters; none of them is part of the inputs' definition)
    solver: dict = field(default_factory=dict)

    @property
    def n_verts(self) -> int:
        return self.rest_xyz.shape[1]

    @property
    def n_tets(self) -> int:
        return self.tets.shape[1]

    @property
    def n_chambers(self) -> int:
        return int(self.alpha.shape[0])


# ---------------------------------------------------------------------------
# voxel -> Kuhn tets
# ---------------------------------------------------------------------------

def kuhn_tets(solid: np.ndarray, h: float, origin=(0.0, 0.0, 0.0)):
    """Split the solid voxels of a boolean grid [nx,ny,nz] into Kuhn tets.

    Returns (xyz [3,n] float64, tets [4,T] int32, voxel_ijk [T,3] int32,
    grid_index [n] int64 of each kept vertex).
    """
    solid = np.asarray(solid, dtype=bool)
    nx, ny, nz = solid.shape
    vox = np.argwhere(solid)                       # lexicographic (i,j,k) order
    nv = vox.shape[0]
    gy, gz = ny + 1, nz + 1

    def gid(ijk):
        return (ijk[..., 0] * gy + ijk[..., 1]) * gz + ijk[..., 2]

    corners = np.empty((nv, 6, 4), dtype=np.int64)
    for p, perm in enumerate(_PERMS):
        e1 = np.zeros(3, dtype=np.int64)
        e1[perm[0]] = 1
        e2 = e1.copy()
        e2[perm[1]] = 1
        offs = [np.zeros(3, dtype=np.int64), e1, e2, np.ones(3, dtype=np.int64)]
        for c, off in enumerate(offs):
            corners[:, p, c] = gid(vox + off)
    flat = corners.reshape(-1, 4)                  # tets in voxel order
    used = np.unique(flat)                         # sorted grid ids = lexicographic
    remap = np.full((nx + 1) * gy * gz, -1, dtype=np.int64)
    remap[used] = np.arange(used.size)
    tets = remap[flat].T.astype(np.int32).copy()
    gi = used // (gy * gz)
    gj = (used // gz) % gy
    gk = used % gz
    xyz = np.stack([gi, gj, gk]).astype(np.float64) * h
    xyz += np.asarray(origin, dtype=np.float64)[:, None]
    voxel_ijk = np.repeat(vox, 6, axis=0).astype(np.int32)
    return xyz, tets, voxel_ijk, used


def _wall_tags(solid: np.ndarray, cavity_id: np.ndarray, gap_side_x: np.ndarray):
    """Per-voxel chamber id (-1 none) and gap-side flag for cavity-wall voxels.

    A cavity-wall voxel is a solid voxel sharing a face with a cavity voxel;
    all 6 of its tets become chamber elements of that cavity's chamber.
    ``gap_side_x[c]`` is a pair (low-x wall faces a slit, high-x wall faces a
    slit) for chamber c; a wall voxel that touches its cavity across an x-face
    in such a wall is gap-side.
    """
    nx, ny, nz = solid.shape
    cham = np.full(solid.shape, -1, dtype=np.int32)
    gap = np.zeros(solid.shape, dtype=bool)
    for axis in range(3):
        for step in (-1, 1):
            nb = np.full(solid.shape, -1, dtype=np.int32)
            src = [slice(None)] * 3
            dst = [slice(None)] * 3
            if step == 1:
                dst[axis] = slice(0, solid.shape[axis] - 1)
                src[axis] = slice(1, None)
            else:
                dst[axis] = slice(1, None)
                src[axis] = slice(0, solid.shape[axis] - 1)
            nb[tuple(dst)] = cavity_id[tuple(src)]
            hit = solid & (nb >= 0)
            cham[hit] = nb[hit]
            if axis == 0:
                # step=+1: cavity lies at higher x -> this voxel is in the cavity's low-x wall
                side = 0 if step == 1 else 1
                flags = np.array([g[side] for g in gap_side_x] + [False])
                gap |= hit & flags[nb]
    return cham, gap


def finger_voxels(h: float, n_chambers: int):
    """Voxel grid of the multi-chamber bending finger (length along x).

    Layout rule (in voxels; r = Python round): ny = nz = r(20/h); root r(6/h);
    chamber block r(12/h); slit max(1,r(1/h)); tip max(1,r(4/h)); base layer
    max(1,r(4/h)) solid along the whole length; cavity walls x r(2/h), sides
    r(4/h), floor r(2/h) above the base, roof r(4/h), each >= 1; slits are
    empty from the top of the base to the top across the full width.
    """
    r = lambda v: max(1, int(round(v)))
    ny = nz = int(round(20.0 / h))
    root = int(round(6.0 / h))
    block = int(round(12.0 / h))
    slit = r(1.0 / h)
    tip = r(4.0 / h)
    base = r(4.0 / h)
    xw, sw, floor, roof = r(2.0 / h), r(4.0 / h), r(2.0 / h), r(4.0 / h)
    c = n_chambers
    nx = root + c * block + (c - 1) * slit + tip
    solid = np.ones((nx, ny, nz), dtype=bool)
    cavity_id = np.full((nx, ny, nz), -1, dtype=np.int32)
    for i in range(c):
        x0 = root + i * (block + slit)
        cx = slice(x0 + xw, x0 + block - xw)
        cy = slice(sw, ny - sw)
        cz = slice(base + floor, nz - roof)
        solid[cx, cy, cz] = False
        cavity_id[cx, cy, cz] = i
        if i < c - 1:
            xs = x0 + block
            solid[xs:xs + slit, :, base:] = False
    gap_side = [(i > 0, i < c - 1) for i in range(c)]
    cham, gap = _wall_tags(solid, cavity_id, gap_side)
    dims = dict(nx=nx, ny=ny, nz=nz, root=root, block=block, slit=slit, tip=tip,
                base=base, xw=xw, sw=sw, floor=floor, roof=roof)
    return solid, cham, gap, dims


def _tags_from_voxels(voxel_ijk, cham, gap, aniso_mode=CH_AX_X):
    vi = voxel_ijk
    c = cham[vi[:, 0], vi[:, 1], vi[:, 2]]
    g = gap[vi[:, 0], vi[:, 1], vi[:, 2]]
    mode = np.where(c >= 0, np.where(g, aniso_mode, CH_ISO), BODY).astype(np.uint8)
    return mode, c.astype(np.int16)


def finger_tet_count(h: float, n_chambers: int) -> int:
    solid, _, _, _ = finger_voxels(h, n_chambers)
    return 6 * int(solid.sum())


def finger(h: float = 2.0, n_chambers: int = 8, alpha=2.0, name=None,
           aniso=True, self_collision=True, precision=4) -> Workload:
    """Multi-chamber bending finger; root face x = 0 is fixed."""
    solid, cham, gap, dims = finger_voxels(h, n_chambers)
    xyz, tets, vijk, _ = kuhn_tets(solid, h)
    mode, chamber = _tags_from_voxels(vijk, cham, gap if aniso else np.zeros_like(gap))
    fixed = (xyz[0] == 0.0).astype(np.uint8)
    a = np.broadcast_to(np.asarray(alpha, dtype=np.float64), (n_chambers,)).copy()
    return Workload(name=name or f"finger_h{h}_c{n_chambers}", rest_xyz=xyz, tets=tets,
                    tet_mode=mode, tet_chamber=chamber, fixed=fixed, alpha=a,
                    self_collision=self_collision, precision=precision,
                    info=dict(h=h, dims=dims))


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def block(h: float = 4.0) -> Workload:
    """Single-chamber block: 100x40x40 mm box, 80x20x20 mm cavity at voxel
    offset (2,2,2) (sizes in units of 4 mm voxels: 25x10x10 with a 20x5x5
    cavity), isotropic chamber, alpha = 1.5, z = 0 face fixed, no collision,
    FP64, 50 fixed iterations."""
    s = 4.0 / h
    nx, ny, nz = int(round(25 * s)), int(round(10 * s)), int(round(10 * s))
    solid = np.ones((nx, ny, nz), dtype=bool)
    cavity = np.full(solid.shape, -1, dtype=np.int32)
    o = int(round(2 * s))
    sl = (slice(o, o + int(round(20 * s))), slice(o, o + int(round(5 * s))),
          slice(o, o + int(round(5 * s))))
    solid[sl] = False
    cavity[sl] = 0
    cham, gap = _wall_tags(solid, cavity, [(False, False)])
    xyz, tets, vijk, _ = kuhn_tets(solid, h)
    mode, chamber = _tags_from_voxels(vijk, cham, gap)
    fixed = (xyz[2] == 0.0).astype(np.uint8)
    return Workload(name="block", rest_xyz=xyz, tets=tets, tet_mode=mode,
                    tet_chamber=chamber, fixed=fixed, alpha=np.array([1.5]),
                    precision=8, fixed_iters=50, info=dict(h=h))


# Settings of the accelerated solve for the gripper: its slowest mode (the
# fingertips sliding along each other on frictionless contacts) contracts at
# about 0.9998 per plain iteration, so the Anderson steps extrapolate far
# along it and need accurate global steps (inner tolerance tightened with the
# outer residual down to 1e-6, CG cap 2000), a memory of 16 and only the
# active-set guard (aa_guard 4: GS_AA_GUARD_SET).
GRIPPER_SOLVER = dict(aa_m=16, aa_guard=4, pcg_eta_min=1e-6, pcg_max=2000)


def gripper(h: float = 1.2, seed: int = 3, radius: float = 45.0) -> Workload:
    """Three fingers on a palm (z = 0), angles 0/120/240 deg, pointing -z, the
    base layer facing the axis; sphere r = 30 at (0,0,-95); plane z = -125
    with normal +z; per-finger alpha ~ U[1, 2.5] (seed 3) broadcast to its
    8 chambers; robot-robot and robot-obstacle collision."""
    solid, cham, gap, dims = finger_voxels(h, 8)
    lxyz, ltets, vijk, _ = kuhn_tets(solid, h)
    mode, chamber = _tags_from_voxels(vijk, cham, gap)
    W = dims["ny"] * h
    xyzs, tets, modes, chambers, fixed = [], [], [], [], []
    off = 0
    for f in range(3):
        th = math.radians(120.0 * f)
        rhat = np.array([math.cos(th), math.sin(th), 0.0])
        that = np.array([-math.sin(th), math.cos(th), 0.0])
        zhat = np.array([0.0, 0.0, 1.0])
        # local (x, y, z) -> world: -x along zhat, y along that, z along rhat
        # (a right-handed frame, so tet orientation is preserved).
        w = (radius * rhat[:, None] - lxyz[0][None, :] * zhat[:, None]
             + (lxyz[1] - W / 2)[None, :] * that[:, None]
             + (lxyz[2] - W / 2)[None, :] * rhat[:, None])
        xyzs.append(w)
        tets.append(ltets + off)
        modes.append(mode)
        chambers.append(np.where(chamber >= 0, chamber + 8 * f, -1).astype(np.int16))
        fixed.append((lxyz[0] == 0.0).astype(np.uint8))
        off += lxyz.shape[1]
    rng = np.random.default_rng(seed)
    af = rng.uniform(1.0, 2.5, 3)
    alpha = np.repeat(af, 8)
    return Workload(name="gripper", rest_xyz=np.concatenate(xyzs, axis=1),
                    tets=np.concatenate(tets, axis=1).astype(np.int32),
                    tet_mode=np.concatenate(modes), tet_chamber=np.concatenate(chambers),
                    fixed=np.concatenate(fixed), alpha=alpha,
                    spheres=np.array([[0.0, 0.0, -95.0, 30.0]]),
                    planes=np.array([[0.0, 0.0, -125.0, 0.0, 0.0, 1.0]]),
                    self_collision=True, obstacle_collision=True, precision=4,
                    info=dict(h=h, finger_alpha=af, dims=dims, verts_per_finger=lxyz.shape[1]),
                    solver=GRIPPER_SOLVER)


# ---------------------------------------------------------------------------
# Triangle-mesh obstacles (closed, outward-oriented)
# ---------------------------------------------------------------------------

def _orient_outward(V, F):
    """Wind every triangle of a convex mesh so its normal points away from
    the mesh's vertex centroid."""
    cen = V.mean(axis=1)
    a, b, c = V[:, F[:, 0]], V[:, F[:, 1]], V[:, F[:, 2]]
    n = np.cross((b - a).T, (c - a).T).T
    flip = np.einsum("ij,ij->j", n, (a + b + c) / 3.0 - cen[:, None]) < 0
    F = F.copy()
    F[flip, 1], F[flip, 2] = F[flip, 2].copy(), F[flip, 1].copy()
    return F


def box_mesh(lo, hi):
    """The box [lo, hi] as 12 triangles: verts [3, 8], tris [12, 3]."""
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    V = np.array([[(hi if (i >> k) & 1 else lo)[k] for k in range(3)] for i in range(8)]).T
    quads = [(0, 2, 6, 4), (1, 3, 7, 5), (0, 1, 5, 4), (2, 3, 7, 6), (0, 1, 3, 2), (4, 5, 7, 6)]
    F = np.array([t for q in quads for t in ((q[0], q[1], q[2]), (q[0], q[2], q[3]))], dtype=np.int64)
    return V, _orient_outward(V, F)


def icosphere(center, radius, levels=2):
    """Sphere of the given radius as a subdivided icosahedron (20 * 4^levels
    triangles, vertices on the sphere)."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    P = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
         (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    pts = [np.array(q, float) / np.linalg.norm(q) for q in P]
    for _ in range(levels):
        mid, nf = {}, []

        def m(i, j):
            k = (min(i, j), max(i, j))
            if k not in mid:
                q = pts[i] + pts[j]
                pts.append(q / np.linalg.norm(q))
                mid[k] = len(pts) - 1
            return mid[k]

        for a, b, c in F:
            ab, bc, ca = m(a, b), m(b, c), m(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = nf
    V = np.asarray(center, float)[:, None] + radius * np.array(pts).T
    return V, _orient_outward(V, np.array(F, dtype=np.int64))


# Chamber unit of the membrane rig, in voxels: footprint, height, wall,
# floor and roof thickness.  The full unit holds 13*13*10 - 7*7*5 = 1,445
# solid voxels, i.e. 8,670 tets, the per-chamber count of the paper's
# membrane model (Table I); the coarse one is for quick checks.
MEMBRANE_UNIT = dict(full=dict(side=13, height=10, wall=3, floor=2, roof=3),
                     coarse=dict(side=7, height=5, wall=2, floor=1, roof=1))


def membrane(h: float = 8.0, seed: int = 6, coarse: bool = False, size: float = 250.0) -> Workload:
    """Soft membrane over four chambers (Section IV, membrane case).

    A one-voxel-thick square sheet of side ``size`` mm, its rim fixed, hangs
    half a voxel above a 2 x 2 array of separate chamber units whose floors
    (z = 0) are fixed.  Each unit is a voxel box around one closed cavity; the
    voxels that share a face with the cavity are its chamber elements
    (isotropic), the rest body.  Inflating the units (alpha ~ U[2, 3.5] per
    chamber, seed 6) lifts their roofs into the sheet: the bodies interact
    only through contact between different connected components.  Dragon
    Skin 20 (the rig's material), self-collision on, FP32.

    Voxel layout: the sheet covers M = round(size / h) voxels per side, one
    voxel above the units' height H, and is then lowered by h/2 and shifted
    by (0.382 h, 0.236 h) in x and y; the units
    (side U) sit 2U + g wide with g = max(1, round(16 / h)) voxels between
    them, centred under the sheet; cavities are centred in x and y.
    """
    u = MEMBRANE_UNIT["coarse" if coarse else "full"]
    if coarse:
        h = max(h, 16.0)
    U, H, w, fl, rf = u["side"], u["height"], u["wall"], u["floor"], u["roof"]
    M = int(round(size / h))
    g = max(1, int(round(16.0 / h)))
    o = (M - (2 * U + g)) // 2
    if o < 0:
        raise ValueError("the chamber units do not fit under the sheet")
    nz = H + 2
    solid = np.zeros((M, M, nz), dtype=bool)
    cavity = np.full(solid.shape, -1, dtype=np.int32)
    for c, (i, j) in enumerate(((0, 0), (1, 0), (0, 1), (1, 1))):
        x0, y0 = o + i * (U + g), o + j * (U + g)
        solid[x0:x0 + U, y0:y0 + U, 0:H] = True
        cs = (slice(x0 + w, x0 + U - w), slice(y0 + w, y0 + U - w), slice(fl, H - rf))
        solid[cs] = False
        cavity[cs] = c
    solid[:, :, H + 1] = True                      # the sheet, one voxel above the units
    cham, gap = _wall_tags(solid, cavity, [(False, False)] * 4)
    xyz, tets, vijk, _ = kuhn_tets(solid, h)
    mode, chamber = _tags_from_voxels(vijk, cham, gap)
    top = (H + 1) * h
    on_sheet = xyz[2] >= top
    rim = on_sheet & ((xyz[0] == 0.0) | (xyz[0] == M * h) | (xyz[1] == 0.0) | (xyz[1] == M * h))
    fixed = ((xyz[2] == 0.0) | rim).astype(np.uint8)
    # half a voxel of clearance above the roofs; the sheet's lattice is also
    # shifted off the units' (by 0.382 h and 0.236 h), so that no roof vertex
    # sits exactly under a sheet vertex or edge (an exact tie between
    # triangles for the inverse-normal ray, decided by rounding)
    xyz[0, on_sheet] += 0.382 * h
    xyz[1, on_sheet] += 0.236 * h
    xyz[2, on_sheet] -= 0.5 * h
    rng = np.random.default_rng(seed)
    alpha = rng.uniform(2.0, 3.5, 4)
    sheet = int(np.count_nonzero(vijk[:, 2] == H + 1))
    return Workload(name="membrane_coarse" if coarse else "membrane", rest_xyz=xyz, tets=tets,
                    tet_mode=mode, tet_chamber=chamber, fixed=fixed, alpha=alpha,
                    self_collision=True, precision=4, material=DRAGON_SKIN_20,
                    info=dict(h=h, sheet_voxels=M, unit=dict(u), unit_tets=(tets.shape[1] - sheet) // 4,
                              sheet_tets=sheet))


def batched_specs(n_mesh: int = 256, seed: int = 4):
    """Per-mesh (h, n_chambers, alpha[]) for the uneven batch.

    For each mesh draw T ~ exp(U[ln 5e3, ln 6e4]), c = floor(exp(U[ln 4, ln 13]))
    and c volume ratios U[1, 2.5] (in that order); h is the value in
    {1.00, 1.05, ..., 4.00} mm whose finger tet count is closest to T.
    """
    rng = np.random.default_rng(seed)
    hs = np.round(np.arange(1.0, 4.0 + 1e-9, 0.05), 2)
    cache = {}
    out = []
    for _ in range(n_mesh):
        T = math.exp(rng.uniform(math.log(5e3), math.log(6e4)))
        c = int(math.floor(math.exp(rng.uniform(math.log(4.0), math.log(13.0)))))
        a = rng.uniform(1.0, 2.5, c)
        if c not in cache:
            cache[c] = np.array([finger_tet_count(float(hh), c) for hh in hs])
        counts = cache[c]
        j = int(np.argmin(np.abs(counts - T)))
        out.append(dict(h=float(hs[j]), n_chambers=c, alpha=a, T_draw=T, T=int(counts[j])))
    return out


def batched(n_mesh: int = 256, seed: int = 4, specs=None):
    """List of finger workloads of uneven size (self-collision on, FP32)."""
    specs = specs or batched_specs(n_mesh, seed)
    return [finger(s["h"], s["n_chambers"], s["alpha"], name=f"batch{i}")
            for i, s in enumerate(specs)]


def adjoint_targets(wl: Workload, seed: int = 5, per_finger: int = 10, radius: float = 10.0):
    """Loss vertices and target points for the gripper gradient workload.

    For each finger, the ``per_finger`` tip-face (local x = max) vertices
    nearest the tip-face centre (ties to the lower id); targets are
    X0[v] + radius * u with u uniform in the unit ball (normal direction
    times U^(1/3), seed 5).
    """
    nvf = wl.info["verts_per_finger"]
    verts = []
    for f in range(3):
        lo = f * nvf
        X = wl.rest_xyz[:, lo:lo + nvf]
        # the finger points -z: its tip face is where world z is minimal
        zmin = X[2].min()
        tip = np.nonzero(np.abs(X[2] - zmin) < 1e-9)[0]
        ctr = X[:, tip].mean(axis=1)
        d = np.linalg.norm(X[:, tip] - ctr[:, None], axis=0)
        order = np.lexsort((tip, np.round(d, 9)))
        verts.extend((tip[order[:per_finger]] + lo).tolist())
    verts = np.asarray(verts, dtype=np.int64)
    rng = np.random.default_rng(seed)
    g = rng.normal(size=(verts.size, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    u = rng.uniform(size=verts.size) ** (1.0 / 3.0)
    y = wl.rest_xyz[:, verts].T + radius * g * u[:, None]
    return verts, y


def finger_tip_targets(wl: Workload, seed: int = 5, n: int = 10, radius: float = 10.0):
    """Loss vertices and targets for a single finger (tip face at x = max):
    the ``n`` tip-face vertices nearest the tip-face centre (ties to the lower
    id), targets X0[v] + radius * u with u uniform in the unit ball (seed 5),
    the single-finger form of ``adjoint_targets``."""
    X = wl.rest_xyz
    xmax = X[0].max()
    tip = np.nonzero(np.abs(X[0] - xmax) < 1e-9)[0]
    ctr = X[:, tip].mean(axis=1)
    d = np.linalg.norm(X[:, tip] - ctr[:, None], axis=0)
    order = np.lexsort((tip, np.round(d, 9)))
    verts = tip[order[:n]].astype(np.int64)
    rng = np.random.default_rng(seed)
    g = rng.normal(size=(verts.size, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    u = rng.uniform(size=verts.size) ** (1.0 / 3.0)
    y = X[:, verts].T + radius * g * u[:, None]
    return verts, y


CONFIGS = {
    "block": lambda: block(),
    "finger": lambda: finger(2.0, 8, 2.0, name="finger"),
    "gripper": lambda: gripper(),
    "membrane": lambda: membrane(),
}


def make(name: str) -> Workload:
    return CONFIGS[name]()
