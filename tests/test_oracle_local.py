"""Pins for the oracle's local step (Section III-A; Eqs. 1, 2, 6, 7).

Each check compares the oracle with something other than itself: a property
the paper states, a closed form, or a library routine in a special case.
"""
import numpy as np
import pytest
import scipy.linalg
import torch
from scipy.spatial.transform import Rotation

from paper_2203_02054_amd import meshgen as mg
import oracle
from oracle.local import kabsch, gather_elements
from tests.meshes import voxel_box, random_rotation


def _prob(mesh, **kw):
    nch = int(max(1, mesh["tet_chamber"].max() + 1))
    return oracle.Problem(mesh["rest_xyz"], mesh["tets"], mesh["tet_mode"], mesh["tet_chamber"],
                          mesh["fixed"], nch, oracle.Params(**kw))


def _vol(Tt):
    d = Tt[:, :, 1:] - Tt[:, :, :1]
    return np.linalg.det(d) / 6.0


def test_rest_state_targets_are_rest_shape():
    """alpha = 1 at x = X0: R = I, lambda = 1, w = 1, so T_e = X_e N (Eq. 1 zero)."""
    wl = mg.make("block")
    prob = oracle.Problem.from_workload(wl)
    Tt = oracle.local_step(prob, prob.X0, np.ones(1))
    np.testing.assert_allclose(Tt, prob.P, atol=1e-12 * prob.h_ref)
    assert oracle.energy(prob, prob.X0, Tt) < 1e-20


@pytest.mark.parametrize("mode", [mg.CH_ISO, mg.CH_AX_X, mg.CH_AX_Y, mg.CH_AX_Z])
def test_chamber_target_volume_is_alpha_times_rest(mode):
    """Chamber targets reach alpha * Vol(e) (Eq. 2 through v^t = alpha^(1/3) v, Section III-A.1)."""
    mesh = voxel_box(3, 2, 2, h=2.0, mode=mode, chamber=0)
    prob = _prob(mesh)
    rng = np.random.default_rng(0)
    x = prob.X0 + 0.3 * rng.normal(size=prob.X0.shape)
    for alpha in (1.0, 1.5, 2.5):
        Tt = oracle.local_step(prob, x, np.array([alpha]))
        np.testing.assert_allclose(_vol(Tt), alpha * prob.vol, rtol=1e-12)
        # the target is centred (translation removed by N)
        np.testing.assert_allclose(Tt.sum(axis=2), 0.0, atol=1e-12)


def test_body_target_volume_is_rest_volume():
    """Eq. 7 (volume scaling): body targets keep Vol(e) whenever Vol(B) > 0."""
    mesh = voxel_box(3, 3, 2, h=1.0)
    prob = _prob(mesh)
    rng = np.random.default_rng(1)
    x = np.diag([1.3, 0.9, 1.1]) @ prob.X0
    x = x + 0.08 * rng.normal(size=x.shape)
    Tt, aux = oracle.local_step(prob, x, np.ones(1), aux=True)
    ok = aux["VB"] > 0
    assert ok.mean() > 0.9
    np.testing.assert_allclose(_vol(Tt)[ok], prob.vol[ok], rtol=1e-11)
    # inverted blends fall back to the rotated rest shape, whose volume is Vol(e) too
    np.testing.assert_allclose(_vol(Tt), prob.vol, rtol=1e-11)


def test_kabsch_recovers_exact_rotation_and_matches_scipy():
    rng = np.random.default_rng(2)
    for _ in range(20):
        P = rng.normal(size=(3, 4))
        P -= P.mean(axis=1, keepdims=True)
        Q = random_rotation(rng)
        D = Q @ P
        R = kabsch(torch.from_numpy((D @ P.T)[None])).numpy()[0]
        np.testing.assert_allclose(R, Q, atol=1e-12)
        # a non-rigid D: Kabsch must equal scipy's least-squares alignment
        D2 = D + 0.3 * rng.normal(size=D.shape)
        R2 = kabsch(torch.from_numpy((D2 @ P.T)[None])).numpy()[0]
        Rs, _ = Rotation.align_vectors(D2.T, P.T)
        np.testing.assert_allclose(R2, Rs.as_matrix(), atol=1e-10)
        M = D2 @ P.T
        if np.linalg.det(M) > 0:
            U, _ = scipy.linalg.polar(M)
            np.testing.assert_allclose(R2, U, atol=1e-10)


def _mr_ratio(lam, c1, c2):
    """Uniaxial incompressible Mooney-Rivlin nominal stress over its linearisation at lambda = 1."""
    stress = 2.0 * (lam - lam ** -2) * (c1 + c2 / lam)
    lin = 6.0 * (c1 + c2) * (lam - 1.0)
    return stress / lin


@pytest.mark.parametrize("c1,c2", [mg.ECOFLEX_0030, mg.DRAGON_SKIN_20])
def test_weight_is_secant_stiffness_ratio(c1, c2):
    lam = np.array([1.05, 1.1, 1.25, 1.5, 2.0, 3.0, 10.0])
    np.testing.assert_allclose(oracle.mooney_rivlin_weight(lam, c1, c2), _mr_ratio(lam, c1, c2), rtol=1e-12)
    assert oracle.mooney_rivlin_weight(1.0, c1, c2) == pytest.approx(1.0, abs=1e-15)
    assert oracle.mooney_rivlin_weight(1e12, c1, c2) == pytest.approx(c1 / (3 * (c1 + c2)), rel=1e-9)


def test_weight_table_values():
    """Values of R_w at the Section IV material constants (Ecoflex 00-30, Dragon Skin 20)."""
    c1, c2 = mg.ECOFLEX_0030
    for lam, w in [(1.1, 0.895077), (1.25, 0.780427), (1.5, 0.656253), (2.0, 0.524332), (3.0, 0.416549)]:
        assert oracle.mooney_rivlin_weight(lam, c1, c2) == pytest.approx(w, abs=1e-6)
    c1, c2 = mg.DRAGON_SKIN_20
    for lam, w in [(1.5, 0.665710), (2.0, 0.536092)]:
        assert oracle.mooney_rivlin_weight(lam, c1, c2) == pytest.approx(w, abs=1e-6)


def test_stretch_measure_uniaxial_and_dilation():
    mesh = voxel_box(1, 1, 1, h=1.0)
    prob = _prob(mesh)
    s = 1.7
    F = np.diag([s, s ** -0.5, s ** -0.5])
    _, aux = oracle.local_step(prob, F @ prob.X0, np.ones(1), aux=True)
    np.testing.assert_allclose(aux["lam"], np.sqrt((s * s + 2.0 / s) / 3.0), rtol=1e-12)
    # pure dilation has Ibar1 = 3: lambda = 1, w = 1, so the target is the rest shape
    Tt, aux = oracle.local_step(prob, 1.4 * prob.X0, np.ones(1), aux=True)
    np.testing.assert_allclose(aux["lam"], 1.0, rtol=1e-12)
    np.testing.assert_allclose(Tt, prob.P, atol=1e-12)


def test_hyperelastic_off_gives_rotated_rest_shape():
    mesh = voxel_box(2, 2, 1, h=1.0)
    prob = _prob(mesh, hyperelastic=False)
    rng = np.random.default_rng(3)
    x = prob.X0 + 0.2 * rng.normal(size=prob.X0.shape)
    Tt, aux = oracle.local_step(prob, x, np.ones(1), aux=True)
    np.testing.assert_allclose(Tt, aux["R"] @ prob.P, atol=1e-12)


def test_local_step_rigid_equivariance():
    """T(Q x + t) = Q T(x) for body and isotropic chamber elements."""
    mesh = voxel_box(3, 2, 2, h=1.0)
    mesh["tet_mode"][::3] = mg.CH_ISO
    mesh["tet_chamber"][::3] = 0
    prob = _prob(mesh)
    rng = np.random.default_rng(4)
    x = prob.X0 + 0.15 * rng.normal(size=prob.X0.shape)
    Q = random_rotation(rng)
    t = rng.normal(size=(3, 1)) * 10
    a = np.array([1.8])
    T1 = oracle.local_step(prob, x, a)
    T2 = oracle.local_step(prob, Q @ x + t, a)
    np.testing.assert_allclose(T2, Q[None] @ T1, atol=1e-11)


def test_gather_elements_layout():
    mesh = voxel_box(1, 1, 1)
    prob = _prob(mesh)
    xe = gather_elements(prob, prob.X0)
    for e in range(prob.T):
        for j in range(4):
            np.testing.assert_array_equal(xe[e, :, j], prob.X0[:, prob.tets[j, e]])
