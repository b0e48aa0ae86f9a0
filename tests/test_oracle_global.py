"""Pins for the oracle's global step and iteration (Section III-B; Eq. 9)."""
import numpy as np
import pytest

from paper_2203_02054_amd import meshgen as mg
import oracle
from oracle import solver
from oracle.collision import Contacts
from tests.meshes import voxel_box, random_rotation


def _prob(mesh, nch=1, **kw):
    return oracle.Problem(mesh["rest_xyz"], mesh["tets"], mesh["tet_mode"], mesh["tet_chamber"],
                          mesh["fixed"], nch, oracle.Params(**kw))


def _grad_eq9(prob, x, Tt, contacts):
    """Gradient of Eq. 9 w.r.t. vertex positions, element by element (no matrix)."""
    g = np.zeros_like(x)
    for e in range(prob.T):
        xe = x[:, prob.tets[:, e]]
        D = xe - xe.mean(axis=1, keepdims=True)
        G = 2.0 * prob.omega[e] * (D - Tt[e])
        # d/dx_e |x_e N - T|^2 = 2 (x_e N - T) N and (D - T) N = D - T (both centred)
        for j in range(4):
            g[:, prob.tets[j, e]] += G[:, j]
    if contacts is not None:
        for s, slot in zip(*np.nonzero(contacts.active)):
            v = prob.query_verts[s]
            g[:, v] += 2.0 * prob.k_spring[v] * (x[:, v] - contacts.target[s, slot])
    return g


def _random_contacts(prob, rng, n=5):
    c = Contacts.empty(prob.query_verts.size, prob.n_slots)
    idx = rng.choice(prob.query_verts.size, size=n, replace=False)
    c.active[idx, 0] = True
    c.target[idx, 0] = prob.X0[:, prob.query_verts[idx]].T + rng.normal(size=(n, 3))
    return c


def test_global_step_is_the_minimiser():
    """The global step zeroes the gradient of Eq. 9 on the free vertices."""
    mesh = voxel_box(3, 2, 2, h=1.0)
    mesh["fixed"][:3] = 1
    prob = _prob(mesh)
    rng = np.random.default_rng(0)
    x = prob.X0 + 0.2 * rng.normal(size=prob.X0.shape)
    x[:, prob.fixed] = prob.X0[:, prob.fixed]
    Tt = oracle.local_step(prob, x, np.ones(1))
    A = _random_contacts(prob, rng)
    xn = oracle.global_step(prob, Tt, A, x)
    g = _grad_eq9(prob, xn, Tt, A)
    assert np.abs(g[:, prob.free]).max() < 1e-10
    np.testing.assert_array_equal(xn[:, prob.fixed], prob.X0[:, prob.fixed])
    # and it is a minimum: random perturbations of free vertices never lower E
    E0 = oracle.energy(prob, xn, Tt, A)
    for _ in range(5):
        d = rng.normal(size=xn.shape) * 1e-3
        d[:, prob.fixed] = 0
        assert oracle.energy(prob, xn + d, Tt, A) >= E0


def test_residual_rhs_is_half_negative_gradient():
    """b - M x (the GPU's correction-form right-hand side) equals -1/2 grad E."""
    mesh = voxel_box(2, 2, 2, h=1.0)
    mesh["fixed"][:2] = 1
    prob = _prob(mesh)
    rng = np.random.default_rng(1)
    x = prob.X0 + 0.1 * rng.normal(size=prob.X0.shape)
    Tt = oracle.local_step(prob, x, np.ones(1))
    A = _random_contacts(prob, rng, 3)
    r = oracle.residual_rhs(prob, x, Tt, A)
    g = _grad_eq9(prob, x, Tt, A)
    g[:, prob.fixed] = 0
    np.testing.assert_allclose(r, -0.5 * g, atol=1e-12)


def test_rest_shape_is_fixed_point_with_zero_energy():
    wl = mg.make("block")
    prob = oracle.Problem.from_workload(wl)
    x, _, st = oracle.solve(prob, np.ones(1), max_iter=3, fixed_iters=0)
    assert st["converged"] and st["iters"] == 1
    assert st["energy"] < 1e-20
    assert np.abs(x - prob.X0).max() < 1e-10 * prob.diag


@pytest.mark.parametrize("alpha", [1.5, 2.0])
def test_all_chamber_box_expands_in_closed_form(alpha):
    """All elements isotropic chamber, one fixed vertex: x = x_f + alpha^(1/3) (X0 - x_f)
    after one iteration, with zero energy afterwards."""
    mesh = voxel_box(3, 2, 2, h=1.0, mode=mg.CH_ISO, chamber=0)
    mesh["fixed"][5] = 1
    prob = _prob(mesh)
    x, _, st = oracle.solve(prob, np.array([alpha]), fixed_iters=1)
    xf = prob.X0[:, 5:6]
    np.testing.assert_allclose(x, xf + alpha ** (1 / 3) * (prob.X0 - xf), atol=1e-12)
    Tt = oracle.local_step(prob, x, np.array([alpha]))
    assert oracle.energy(prob, x, Tt) < 1e-20


def test_arap_energy_decreases_monotonically():
    """With R_w == 1 and a fixed contact set each local and global step is an exact
    block minimisation of Eq. 9, so E_k never increases."""
    wl = mg.finger(4.0, 3, 2.0, self_collision=False)
    prob = oracle.Problem.from_workload(wl, hyperelastic=False)
    _, _, st = oracle.solve(prob, wl.alpha, fixed_iters=25, history=True)
    E = np.array([h["E"] for h in st["history"]])
    assert np.all(np.diff(E) <= 1e-9 * E[0])
    assert E[-1] < 0.5 * E[0]


def test_surrogate_energy_decreases_with_collision_and_hyperelastic_weights():
    """E(x_{k+1}; T_k) <= E(x_k; T_k) always (exact global step)."""
    wl = mg.finger(4.0, 3, 2.0)
    prob = oracle.Problem.from_workload(wl)
    _, _, st = oracle.solve(prob, wl.alpha, fixed_iters=20, history=True)
    for h in st["history"]:
        assert h["E_sur"] <= h["E"] * (1 + 1e-12)


def test_rigid_motion_invariance_of_the_solve():
    """x*(Q X0 + t) = Q x*(X0) + t (no gravity; isotropic chambers only)."""
    wl = mg.finger(4.0, 3, 1.8, aniso=False, self_collision=False)
    p1 = oracle.Problem.from_workload(wl)
    rng = np.random.default_rng(5)
    Q = random_rotation(rng)
    t = np.array([[3.0], [-7.0], [11.0]])
    p2 = oracle.Problem(Q @ wl.rest_xyz + t, wl.tets, wl.tet_mode, wl.tet_chamber, wl.fixed,
                        wl.n_chambers, p1.params)
    x1, _, _ = oracle.solve(p1, wl.alpha, fixed_iters=15)
    x2, _, _ = oracle.solve(p2, wl.alpha, fixed_iters=15)
    np.testing.assert_allclose(x2, Q @ x1 + t, atol=1e-10 * p1.diag)


def test_fixed_vertices_never_move_and_warm_start_resumes():
    wl = mg.finger(4.0, 3, 2.0)
    prob = oracle.Problem.from_workload(wl)
    xa, Aa, _ = oracle.solve(prob, wl.alpha, fixed_iters=12)
    x1, A1, _ = oracle.solve(prob, wl.alpha, fixed_iters=5)
    x2, A2, _ = oracle.solve(prob, wl.alpha, x0=x1, contacts0=A1, fixed_iters=7)
    np.testing.assert_array_equal(xa[:, prob.fixed], prob.X0[:, prob.fixed])
    np.testing.assert_allclose(x2, xa, atol=1e-12 * prob.diag)
    assert A2.same_set(Aa)
