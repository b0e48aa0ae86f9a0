"""The membrane workload on the oracle (Section IV, membrane case): the
coarse rig reaches a fixed point in which the sheet rests on the inflated
chamber units through contacts between different bodies.

These are properties of the oracle's solution that the geometry fixes: the
units' roofs rise by more than the clearance when inflated alone (so without
contact they would pass through the sheet), every sheet-unit contact pairs a
vertex of one body with a face of another, and at the fixed point no query
vertex is left inside an element of another body by more than the offset.
"""
import dataclasses

import numpy as np
import pytest

from paper_2203_02054_amd import meshgen as mg
import oracle
from oracle.collision import SELF
from tests.test_meshgen import _components


@pytest.fixture(scope="module")
def coarse():
    wl = mg.membrane(coarse=True)
    prob = oracle.Problem.from_workload(wl)
    x, c, st = oracle.solve(prob, wl.alpha, max_iter=300, anderson=8)
    return wl, prob, x, c, st


def test_membrane_reaches_a_fixed_point_with_contacts_between_bodies(coarse):
    wl, prob, x, c, st = coarse
    assert st["converged"] and st["residual"] <= 1e-6
    rows, _ = c.listing(prob)
    comp = _components(wl.n_verts, wl.tets)
    self_rows = rows[rows[:, 1] == SELF]
    assert self_rows.shape[0] > 20
    v, f = self_rows[:, 0], self_rows[:, 2]
    across = comp[v] != comp[prob.faces[f, 0]]
    assert across.sum() > 20
    # the sheet is lifted by its contacts
    h = wl.info["h"]
    sheet = prob.X0[2] > wl.info["unit"]["height"] * h + 1e-9
    assert (x[2] - prob.X0[2])[sheet].max() > 0.1 * h


def test_without_contact_the_roofs_would_cross_the_sheet():
    wl = mg.membrane(coarse=True)
    wl0 = dataclasses.replace(wl, self_collision=False)
    prob = oracle.Problem.from_workload(wl0)
    x, _, st = oracle.solve(prob, wl.alpha, max_iter=300, anderson=8)
    assert st["converged"]
    h = wl.info["h"]
    sheet = prob.X0[2] > wl.info["unit"]["height"] * h + 1e-9
    assert x[2, ~sheet].max() > x[2, sheet].min() + 0.1 * h
