"""Pins for the oracle's set-up quantities (Section II-A and the offsets of
Section II-C that derive from the reference length h_ref)."""
import numpy as np
import pytest

import oracle
from tests.meshes import voxel_box


@pytest.mark.parametrize("nx,ny,nz,h", [(1, 1, 1, 1.0), (3, 2, 4, 2.5)])
def test_h_ref_is_the_mean_of_the_unique_edges_of_a_kuhn_box(nx, ny, nz, h):
    """h_ref is the mean rest length of the unique tet edges.  In a full
    nx x ny x nz box of Kuhn-split voxels of size h these are the grid's axis
    edges (length h), one diagonal per grid square (h sqrt 2) and one body
    diagonal per voxel (h sqrt 3), counted in closed form.  A mean over the
    edges of every tet, shared ones repeated (3 axis, 2 face and 1 body
    diagonal per tet), would give h (3 + 2 sqrt 2 + sqrt 3) / 6 instead."""
    mesh = voxel_box(nx, ny, nz, h=h)
    prob = oracle.Problem(mesh["rest_xyz"], mesh["tets"], mesh["tet_mode"], mesh["tet_chamber"],
                          mesh["fixed"], 1, oracle.Params())
    e1 = nx * (ny + 1) * (nz + 1) + (nx + 1) * ny * (nz + 1) + (nx + 1) * (ny + 1) * nz
    e2 = nx * ny * (nz + 1) + nx * (ny + 1) * nz + (nx + 1) * ny * nz
    e3 = nx * ny * nz
    expected = h * (e1 + np.sqrt(2.0) * e2 + np.sqrt(3.0) * e3) / (e1 + e2 + e3)
    assert prob.h_ref == pytest.approx(expected, rel=1e-14)
    per_tet_mean = h * (3.0 + 2.0 * np.sqrt(2.0) + np.sqrt(3.0)) / 6.0
    assert abs(prob.h_ref - per_tet_mean) > 0.01 * h
    # the offsets that the collision response derives from it (defaults)
    assert prob.eps_off == pytest.approx(0.05 * expected, rel=1e-14)
