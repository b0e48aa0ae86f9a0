"""Pins for the oracle's remesh checks and progressive actuation (Section
III-B; Algorithm 1's outer loop).

Affine deformations x = F X0 + t give every element the same deformation
gradient F, so each element's volume ratio is det F and its distortion
norm(Sigma) is 1/sigma_min(F) in closed form.  The cases are chosen so that a
plausible slip fails one of them: using F instead of its inverse (the
stretch diag(5,1,1) would then read as distorted), the inverse volume ratio
(diag(5,1,1) would read 0.2), flagging body elements, or swapping the
deformed and reference shapes.
"""
import numpy as np
import pytest

from paper_2203_02054_amd import meshgen as mg
import oracle
from oracle import remesh
from tests.meshes import voxel_box, random_rotation


def _finger():
    return oracle.Problem.from_workload(mg.finger(4.0, 3, 2.0))


CASES = [  # singular values of F (in a random frame), volume flag, distortion flag
    ((5.0, 1.0, 1.0), True, False),
    ((1.0, 1.0, 0.2), False, True),
    ((2.0, 2.0, 2.0), True, False),
    ((6.0, 0.2, 1.0), False, True),
    ((25.0, 1.0, 0.2), True, True),
    ((1.5, 1.5, 1.5), False, False),
    ((3.9, 1.0, 0.26), False, False),
]


@pytest.mark.parametrize("sv,vol,dist", CASES)
def test_affine_deformation_measures_and_flags(sv, vol, dist):
    prob = _finger()
    rng = np.random.default_rng(11)
    Q1, Q2 = random_rotation(rng), random_rotation(rng)
    F = Q1 @ np.diag(sv) @ Q2
    x = F @ prob.X0 + rng.normal(size=(3, 1))
    ratio, dn = remesh.remesh_measures(prob, x)
    np.testing.assert_allclose(ratio, np.prod(sv), rtol=1e-10)
    np.testing.assert_allclose(dn, 1.0 / min(sv), rtol=1e-10)
    f = remesh.remesh_flags(prob, x)
    chamber = prob.mode != mg.BODY
    assert chamber.any() and (~chamber).any()
    assert np.all(f[~chamber] == 0)
    expect = (remesh.VOLUME if vol else 0) | (remesh.DISTORTION if dist else 0)
    assert np.all(f[chamber] == expect)


def test_reference_shape_is_the_one_passed():
    """x = F2 (F1 X0) against the reference F1 X0 measures F2 alone."""
    prob = _finger()
    rng = np.random.default_rng(12)
    F1 = random_rotation(rng) @ np.diag([3.0, 0.5, 1.0])
    F2 = random_rotation(rng) @ np.diag([1.0, 6.0, 0.1])
    ref = F1 @ prob.X0
    ratio, dn = remesh.remesh_measures(prob, F2 @ ref, ref)
    np.testing.assert_allclose(ratio, 0.6, rtol=1e-10)
    np.testing.assert_allclose(dn, 10.0, rtol=1e-10)
    # against the rest shape the same positions measure F2 F1
    ratio0, dn0 = remesh.remesh_measures(prob, F2 @ ref)
    np.testing.assert_allclose(ratio0, 0.9, rtol=1e-10)
    np.testing.assert_allclose(dn0, 1.0 / np.linalg.svd(F2 @ F1, compute_uv=False)[-1], rtol=1e-10)


def test_flattened_element_is_infinitely_distorted():
    prob = _finger()
    x = np.diag([1.0, 1.0, 0.0]) @ prob.X0
    ratio, dn = remesh.remesh_measures(prob, x)
    assert np.all(np.abs(ratio) < 1e-12)
    chamber = prob.mode != mg.BODY
    assert np.all(remesh.remesh_flags(prob, x)[chamber] == remesh.DISTORTION)


def test_thresholds_are_parameters_and_strict():
    prob = _finger()
    x = 2.0 * prob.X0                      # ratio 8, norm(Sigma) 0.5
    chamber = prob.mode != mg.BODY
    assert np.all(remesh.remesh_flags(prob, x, alpha_max=9.0)[chamber] == 0)
    assert np.all(remesh.remesh_flags(prob, x, alpha_max=7.0)[chamber] == remesh.VOLUME)
    assert np.all(remesh.remesh_flags(prob, x, alpha_max=9.0, d_max=0.25)[chamber] == remesh.DISTORTION)
    assert np.all(remesh.remesh_flags(prob, x, alpha_max=9.0, d_max=0.5)[chamber] == 0)


def test_local_flag_is_confined_to_the_moved_vertex():
    """Moving one vertex changes only the elements around it (brute force)."""
    prob = _finger()
    chamber = np.nonzero(prob.mode != mg.BODY)[0]
    v = int(prob.tets[0, chamber[len(chamber) // 2]])
    x = prob.X0.copy()
    h = prob.h_ref
    x[:, v] += np.array([0.0, 0.0, 40.0 * h])     # pulls its elements far out
    f = remesh.remesh_flags(prob, x)
    around = np.any(prob.tets == v, axis=0)
    assert np.all(f[~around] == 0)
    assert np.any(f[around & (prob.mode != mg.BODY)] != 0)
    # element by element, with the volume written as a scalar triple product
    for e in np.nonzero(around)[0]:
        a, b, c, d = (x[:, prob.tets[k, e]] for k in range(4))
        A, B, C, D = (prob.X0[:, prob.tets[k, e]] for k in range(4))
        r = np.dot(np.cross(b - a, c - a), d - a) / np.dot(np.cross(B - A, C - A), D - A)
        if prob.mode[e] != mg.BODY:
            assert bool(f[e] & remesh.VOLUME) == (r > 4.0)


def test_stage_schedule():
    st = remesh.stage_alphas(np.array([10.0, 3.0]), 4.0)
    np.testing.assert_array_equal(np.array(st), [[4.0, 3.0], [8.0, 3.0], [10.0, 3.0]])
    assert [list(a) for a in remesh.stage_alphas([2.5], 4.0)] == [[2.5]]
    assert [list(a) for a in remesh.stage_alphas([4.0], 4.0)] == [[4.0]]
    assert [list(a) for a in remesh.stage_alphas([8.0], 4.0)] == [[4.0], [8.0]]
    assert [list(a) for a in remesh.stage_alphas([0.5], 4.0)] == [[0.5]]
    with pytest.raises(ValueError):
        remesh.stage_alphas([np.nan], 4.0)


def test_progressive_all_chamber_box_in_closed_form():
    """All-chamber box, one fixed vertex: every stage ends at
    x_f + alpha_k^(1/3) (X0 - x_f), so after the stages alpha_k = 4, 8, 10 the
    volume ratio is alpha_k exactly; 8 and 10 flag every element for volume,
    none for distortion (sigma = alpha_k^(1/3) in every direction)."""
    mesh = voxel_box(3, 2, 2, h=1.0, mode=mg.CH_ISO, chamber=0)
    mesh["fixed"][5] = 1
    prob = oracle.Problem(mesh["rest_xyz"], mesh["tets"], mesh["tet_mode"], mesh["tet_chamber"],
                          mesh["fixed"], 1, oracle.Params(tol=1e-12))
    xf = prob.X0[:, 5:6]
    x, _, flags, stages = remesh.solve_progressive(prob, np.array([10.0]), stop_on_flag=False)
    assert [float(s["alpha"][0]) for s in stages] == [4.0, 8.0, 10.0]
    np.testing.assert_allclose(x, xf + 10.0 ** (1 / 3) * (prob.X0 - xf), atol=1e-11)
    assert stages[1]["n_flagged"] == prob.T and stages[2]["n_flagged"] == prob.T
    assert np.all(flags == remesh.VOLUME)
    # stop at the first stage that flags: stage 0 ends exactly on the
    # threshold (ratio 4, not above it in exact arithmetic), so the loop stops
    # after stage 0 or 1 depending on the last bit, never later
    _, _, flags2, st2 = remesh.solve_progressive(prob, np.array([10.0]), stop_on_flag=True)
    assert len(st2) in (1, 2) and st2[-1]["n_flagged"] > 0
    assert all(s["n_flagged"] == 0 for s in st2[:-1])
