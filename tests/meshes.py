"""Tiny hand-built meshes shared by the CPU and GPU tests (inputs only)."""
import numpy as np

from paper_2203_02054_amd import meshgen as mg


def voxel_box(nx, ny, nz, h=1.0, mode=mg.BODY, chamber=-1):
    solid = np.ones((nx, ny, nz), bool)
    xyz, tets, _, _ = mg.kuhn_tets(solid, h)
    T = tets.shape[1]
    return dict(rest_xyz=xyz, tets=tets, tet_mode=np.full(T, mode, np.uint8),
                tet_chamber=np.full(T, chamber, np.int16),
                fixed=np.zeros(xyz.shape[1], np.uint8))


def slit_pair(h=1.0, gap=1, depth=2):
    """Two voxel blocks facing each other across an empty slab (a slit)."""
    nx = 2 * depth + gap
    solid = np.ones((nx, 2, 2), bool)
    solid[depth:depth + gap] = False
    xyz, tets, vijk, _ = mg.kuhn_tets(solid, h)
    T = tets.shape[1]
    return dict(rest_xyz=xyz, tets=tets, tet_mode=np.zeros(T, np.uint8),
                tet_chamber=np.full(T, -1, np.int16),
                fixed=np.zeros(xyz.shape[1], np.uint8)), vijk


def random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def pressed_finger():
    """A small finger (h = 4 mm, 3 chambers, alpha 2) with a sphere above its
    tip and a plane 0.6 mm above its base face: its iterations carry self
    contacts with new ray targets, kept self contacts, sphere and plane
    contacts."""
    import dataclasses
    w = mg.finger(4.0, 3, 2.0)
    X = w.rest_xyz
    sph = np.array([[X[0].max() - 8.0, 10.0, X[2].max() + 3.0, 6.0]])
    pl = np.array([[0.0, 0.0, 0.6, 0.0, 0.0, 1.0]])
    return dataclasses.replace(w, spheres=sph, planes=pl, obstacle_collision=True, self_collision=True)


def wavy_positions(X, rng, amp, waves=6, noise=0.0):
    """Rest positions X [3,n] moved by a sum of random sinusoidal fields (and
    optional per-vertex noise), all scaled by amp: seeded deformed states
    with a spread of local stretches, squashes and inversions."""
    ext = X.max(axis=1) - X.min(axis=1)
    u = np.zeros_like(X)
    for _ in range(waves):
        k = rng.normal(size=3) * (2 * np.pi / np.maximum(ext, 1e-9))
        ph = rng.uniform(0, 2 * np.pi)
        d = rng.normal(size=3)
        u += d[:, None] * np.sin(k @ X + ph)[None, :]
    u *= amp / np.sqrt(waves)
    if noise:
        u += noise * rng.normal(size=X.shape)
    return X + u
