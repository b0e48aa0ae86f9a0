"""Pins for the oracle's implicit gradient (oracle.adjoint): the polar
derivative against finite differences, the closed-form gradient of an
all-chamber mesh, every part of db/dx against finite differences at a state
with new self contacts, sphere and plane contacts, and the implicit gradient
against central differences of the frozen-set fixed point."""
import numpy as np
import pytest
import torch

from paper_2203_02054_amd import meshgen as mg
import oracle
from oracle import adjoint as oa
from oracle import collision as oc
from oracle import solver as so
from oracle.collision import Contacts
from tests.meshes import pressed_finger, voxel_box


def test_polar_rotation_derivative_matches_finite_differences():
    """M = U diag(s) V^T with distinct |s|, half with det M < 0 (the Kabsch
    reflection case, where R is not the polar factor of M's SVD)."""
    g = torch.Generator().manual_seed(0)
    U = torch.linalg.qr(torch.randn((6, 3, 3), dtype=torch.float64, generator=g))[0]
    V = torch.linalg.qr(torch.randn((6, 3, 3), dtype=torch.float64, generator=g))[0]
    s = torch.tensor([[3.0, 2.0, 1.0], [2.5, 1.5, 0.7], [4.0, 1.0, 0.5],
                      [3.0, 2.0, -1.0], [2.5, 1.5, -0.7], [4.0, 1.0, -0.5]], dtype=torch.float64)
    U = U * torch.sign(torch.linalg.det(U))[:, None, None]      # proper rotations
    V = V * torch.sign(torch.linalg.det(V))[:, None, None]
    M = U @ torch.diag_embed(s) @ V.transpose(1, 2)
    assert (torch.linalg.det(M[:3]) > 0).all() and (torch.linalg.det(M[3:]) < 0).all()
    M.requires_grad_(True)
    assert torch.autograd.gradcheck(oa.polar_rotation, (M,), eps=1e-6, atol=1e-7, rtol=1e-6)
    with torch.no_grad():
        R = oa.polar_rotation(M)
        np.testing.assert_allclose((R.transpose(1, 2) @ R).numpy(), np.broadcast_to(np.eye(3), (6, 3, 3)),
                                   atol=1e-12)
        assert torch.allclose(torch.linalg.det(R), torch.ones(6, dtype=torch.float64))


def _closed_form_case(mode):
    mesh = voxel_box(3, 2, 2, h=1.0, mode=mode, chamber=0)
    mesh["fixed"][5] = 1
    prob = oracle.Problem(mesh["rest_xyz"], mesh["tets"], mesh["tet_mode"], mesh["tet_chamber"],
                          mesh["fixed"], 1, oracle.Params())
    return prob, prob.X0[:, 5:6]


@pytest.mark.parametrize("mode,alpha", [(mg.CH_ISO, 1.5), (mg.CH_ISO, 2.0), (mg.CH_AX_X, 1.7), (mg.CH_AX_Z, 2.2)])
def test_all_chamber_gradient_in_closed_form(mode, alpha):
    """All elements chamber, one fixed vertex x_f: the fixed point is the
    rest shape scaled about x_f (by alpha^(1/3), or by alpha along the axis),
    so L = sum_v |x_v - x_f|^2 (invariant to the free rotation about x_f) has
    dL/dalpha = (2/3) alpha^(-1/3) sum |X_v - x_f|^2 (isotropic) or
    2 alpha sum (X_v - x_f)_axis^2 (axis)."""
    prob, xf = _closed_form_case(mode)
    s = np.ones((3, 1))
    if mode == mg.CH_ISO:
        s[:] = alpha ** (1.0 / 3.0)
        exact = (2.0 / 3.0) * alpha ** (-1.0 / 3.0) * ((prob.X0 - xf) ** 2).sum()
    else:
        ax = {mg.CH_AX_X: 0, mg.CH_AX_Y: 1, mg.CH_AX_Z: 2}[mode]
        s[ax] = alpha
        exact = 2.0 * alpha * ((prob.X0[ax] - xf[ax]) ** 2).sum()
    xs = xf + s * (prob.X0 - xf)
    A = Contacts.empty(prob.query_verts.size, prob.n_slots)
    fresh = np.zeros(prob.query_verts.size, bool)
    step = oa.frozen_map(prob, xs, np.array([alpha]), A, fresh)
    assert np.abs(step - xs).max() < 1e-12                # it is the fixed point
    ga, _, info = oa.grad(prob, xs, np.array([alpha]), A, fresh, 2.0 * (xs - xf))
    assert info["residual"] < 1e-12
    assert ga[0] == pytest.approx(exact, rel=1e-12)


@pytest.fixture(scope="module")
def contact_state():
    """A small finger (h = 4 mm, 3 chambers) pressed by a sphere and a plane,
    after 61 iterations from rest: the active set holds self contacts with new
    ray targets, kept self contacts, sphere and plane contacts."""
    w = pressed_finger()
    prob = oracle.Problem.from_workload(w)
    x, prev, fac = prob.X0.copy(), None, so._Factor()
    for _ in range(61):
        x, prev, _, _ = so.step(prob, x, w.alpha, prev, fac)
    A, info = oc.collide(prob, x, prev)
    fresh = info["self_fresh"]
    assert fresh.sum() >= 2 and (A.active[:, 0] & ~fresh).any()
    assert A.active[:, 1].any() and A.active[:, 2].any()
    return prob, w, x, A, fresh


@pytest.mark.parametrize("part", ["elements", "new_self", "kept_self", "sphere", "plane"])
def test_rhs_jacobian_matches_finite_differences(contact_state, part):
    prob, w, x, A, fresh = contact_state
    B = A.copy()
    if part == "elements":
        B = Contacts.empty(prob.query_verts.size, prob.n_slots)
    else:
        keep = {"new_self": (0, fresh), "kept_self": (0, ~fresh), "sphere": (1, None), "plane": (2, None)}[part]
        for sl in range(prob.n_slots):
            if sl != keep[0]:
                B.active[:, sl] = False
        if keep[1] is not None:
            B.active[:, 0] &= keep[1]
        assert B.count > 0
    rng = np.random.default_rng(1)
    mu, v = rng.standard_normal((3, prob.n)), rng.standard_normal((3, prob.n))
    al = torch.from_numpy(w.alpha.copy())
    xt = torch.tensor(x, requires_grad=True)
    b = oa.rhs(prob, xt, al, B, fresh)
    (gx,) = torch.autograd.grad(b, xt, grad_outputs=torch.from_numpy(mu))
    h = 1e-5
    with torch.no_grad():
        bp = oa.rhs(prob, torch.from_numpy(x + h * v), al, B, fresh).numpy()
        bm = oa.rhs(prob, torch.from_numpy(x - h * v), al, B, fresh).numpy()
    fd = (mu * (bp - bm)).sum() / (2 * h)
    assert (gx.numpy() * v).sum() == pytest.approx(fd, rel=1e-7)
    if part == "kept_self":
        # a kept self target is a constant: only the spring-free element part moves
        E = Contacts.empty(prob.query_verts.size, prob.n_slots)
        (ge,) = torch.autograd.grad(oa.rhs(prob, xt, al, E, fresh), xt, grad_outputs=torch.from_numpy(mu))
        np.testing.assert_allclose(gx.numpy(), ge.numpy(), atol=1e-12)


def test_implicit_gradient_matches_central_differences(contact_state):
    """dL/dalpha by the implicit function theorem against central differences
    of the frozen-set fixed point, L = g . x with a seeded g.  The step is
    h = 1e-4: the fixed point is only resolved to ~1e-14 diag per solve and the
    map contracts slowly, so with h = 1e-6 the solve error, not the
    derivative, would dominate the difference quotient."""
    prob, w, x, A, fresh = contact_state
    xs, _, step = oa.frozen_solve(prob, w.alpha, x, A, fresh, tol=1e-14)
    assert step <= 1e-14
    rng = np.random.default_rng(0)
    g = rng.standard_normal((3, prob.n))
    g[:, prob.fixed] = 0.0
    ga, _, info = oa.grad(prob, xs, w.alpha, A, fresh, g)
    assert info["residual"] < 1e-12
    h = 1e-4
    fd = np.zeros(w.n_chambers)
    for c in range(w.n_chambers):
        ap, am = w.alpha.copy(), w.alpha.copy()
        ap[c] += h
        am[c] -= h
        xp, _, sp_ = oa.frozen_solve(prob, ap, xs, A, fresh, tol=1e-14)
        xm, _, sm_ = oa.frozen_solve(prob, am, xs, A, fresh, tol=1e-14)
        assert sp_ <= 1e-14 and sm_ <= 1e-14
        fd[c] = ((g * xp).sum() - (g * xm).sum()) / (2 * h)
    assert np.linalg.norm(ga - fd) <= 1e-5 * np.linalg.norm(fd)


def test_unrolled_gradient_matches_central_differences():
    """Unrolled gradient through 30 iterations from rest (new and kept self
    contacts, sphere and plane springs along the way) against central
    differences of the same contact schedule replayed for alpha +- h."""
    w = pressed_finger()
    prob = oracle.Problem.from_workload(w)
    path, xK = oa.record_path(prob, w.alpha, prob.X0, None, 30)
    assert sum(int(f.sum()) for _, _, f in path) > 0
    assert np.abs(oa.replay(prob, w.alpha, path) - xK).max() < 1e-12 * prob.diag * 100
    rng = np.random.default_rng(0)
    g = rng.standard_normal((3, prob.n))
    g[:, prob.fixed] = 0.0
    ga, _ = oa.unrolled_grad(prob, w.alpha, path, g)
    h = 1e-5
    fd = np.zeros(w.n_chambers)
    for c in range(w.n_chambers):
        ap, am = w.alpha.copy(), w.alpha.copy()
        ap[c] += h
        am[c] -= h
        fd[c] = ((g * oa.replay(prob, ap, path)).sum() - (g * oa.replay(prob, am, path)).sum()) / (2 * h)
    assert np.linalg.norm(ga - fd) <= 1e-8 * np.linalg.norm(fd)


def test_unrolled_gradient_closed_form():
    """All-chamber box from rest: one iteration reaches the scaled shape, which
    is then a fixed point for every alpha, so the unrolled gradient of
    L = sum |x - x_f|^2 is the closed form for any K >= 1."""
    prob, xf = _closed_form_case(mg.CH_ISO)
    alpha = np.array([1.8])
    path, xK = oa.record_path(prob, alpha, prob.X0, None, 4)
    ga, _ = oa.unrolled_grad(prob, alpha, path, 2.0 * (xK - xf))
    exact = (2.0 / 3.0) * alpha[0] ** (-1.0 / 3.0) * ((prob.X0 - xf) ** 2).sum()
    assert ga[0] == pytest.approx(exact, rel=1e-10)
