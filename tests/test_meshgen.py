"""Synthetic workload generator: element counts and structure.

The expected counts are those of the voxel rule applied to the stated
dimensions (finger/block/gripper layouts); they are independent of both the
oracle and the GPU path.  Surface and CSR counts go through the oracle's
set-up, pinning its boundary extraction and its system assembly pattern.
"""
import numpy as np
import pytest

from paper_2203_02054_amd import meshgen as mg
import oracle

# T, n, surface verts, surface tris, CSR nnz, fixed, wall tets, gap-side tets, chambers
TABLE = {
    "block": (12000, 2842, 1654, 3300, 35822, 286, 2700, 0, 1),
    "finger": (26880, 6901, 4810, 9584, 84029, 121, 7104, 2520, 8),
}


@pytest.mark.parametrize("name", sorted(TABLE))
def test_counts(name):
    wl = mg.make(name)
    T, n, S, F, nnz, fixed, wall, gap, nch = TABLE[name]
    assert wl.n_tets == T and wl.n_verts == n
    assert int(wl.fixed.sum()) == fixed
    assert int((wl.tet_mode > 0).sum()) == wall
    assert int((wl.tet_mode == mg.CH_AX_X).sum()) == gap
    assert wl.n_chambers == nch
    prob = oracle.Problem.from_workload(wl)
    assert prob.surf_verts.size == S
    assert prob.faces.shape[0] == F
    assert prob.A_el.nnz == nnz


def test_gripper_counts():
    wl = mg.gripper()
    assert wl.n_tets == 378666 and wl.n_verts == 83712
    assert int(wl.fixed.sum()) == 3 * 324
    assert int((wl.tet_mode > 0).sum()) == 63072
    assert int((wl.tet_mode == mg.CH_AX_X).sum()) == 24948
    assert wl.n_chambers == 24
    # per-finger actuation from seed 3, broadcast to the finger's 8 chambers
    a = np.random.default_rng(3).uniform(1.0, 2.5, 3)
    np.testing.assert_array_equal(wl.alpha, np.repeat(a, 8))


def test_kuhn_split_conforming_and_volume():
    solid = np.ones((3, 2, 2), bool)
    h = 1.5
    xyz, tets, _, _ = mg.kuhn_tets(solid, h)
    assert tets.shape == (4, 6 * 12)
    # every interior face is shared by exactly two tets, total volume is the box
    P = xyz[:, tets]
    d = P[:, 1:] - P[:, :1]
    vol = np.abs(np.linalg.det(np.moveaxis(d, 2, 0).transpose(0, 2, 1))) / 6
    assert np.isclose(vol.sum(), 12 * h ** 3)
    prob = oracle.Problem(xyz, tets, np.zeros(72, np.uint8), -np.ones(72, np.int16),
                          np.zeros(xyz.shape[1], np.uint8), 0)
    # boundary of a 3x2x2 box: 2*(3*2 + 3*2 + 2*2) squares, 2 triangles each
    assert prob.faces.shape[0] == 2 * 2 * (6 + 6 + 4)


def test_batched_specs_deterministic():
    s1 = mg.batched_specs(8, seed=4)
    s2 = mg.batched_specs(8, seed=4)
    for a, b in zip(s1, s2):
        assert a["h"] == b["h"] and a["n_chambers"] == b["n_chambers"]
        np.testing.assert_array_equal(a["alpha"], b["alpha"])
        assert 4 <= a["n_chambers"] <= 12
        assert np.all((a["alpha"] >= 1.0) & (a["alpha"] <= 2.5))


def _components(n, tets):
    """Connected components of the tet graph (union-find over tet vertices)."""
    parent = np.arange(n)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for t in tets.T:
        r = [find(int(v)) for v in t]
        for q in r[1:]:
            parent[find(q)] = find(r[0])
    return np.array([find(v) for v in range(n)])


@pytest.mark.parametrize("coarse", [False, True])
def test_membrane_layout(coarse):
    """Four chamber units of 13*13*10 - 7*7*5 = 1,445 voxels (8,670 tets each,
    Table I's per-chamber count) or 7*7*5 - 3*3*3 = 218 voxels (coarse), one
    wall layer of chamber elements around each cavity, and a one-voxel sheet
    of M*M voxels; floors and the sheet's rim fixed; five separate bodies."""
    wl = mg.membrane(coarse=coarse)
    h = wl.info["h"]
    M = wl.info["sheet_voxels"]
    unit_vox, cav, wall_vox, side = ((218, (3, 3, 3), 2 * 9 + 4 * 9, 7) if coarse
                                     else (1445, (7, 7, 5), 2 * 49 + 4 * 35, 13))
    assert wl.info["unit_tets"] == 6 * unit_vox
    assert wl.n_tets == 4 * 6 * unit_vox + 6 * M * M
    if not coarse:
        assert 4 * wl.info["unit_tets"] == 34680
    assert wl.n_chambers == 4
    for c in range(4):
        assert int((wl.tet_chamber == c).sum()) == 6 * wall_vox
    assert np.all(wl.tet_mode[wl.tet_mode > 0] == mg.CH_ISO)
    assert int(wl.fixed.sum()) == 4 * (side + 1) ** 2 + 2 * 4 * M
    comp = _components(wl.n_verts, wl.tets)
    assert np.unique(comp).size == 5
    X = wl.rest_xyz
    sheet = X[2] > wl.info["unit"]["height"] * h + 1e-9
    assert X[2, sheet].min() - X[2, ~sheet].max() == pytest.approx(0.5 * h)
    assert np.all(1.5 <= wl.alpha) and np.all(wl.alpha <= 3.5)
