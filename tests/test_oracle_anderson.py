"""Pins for the oracle's Anderson-accelerated local/global iteration (the
acceleration the paper applies to its solver, end of Section III-B; Walker &
Ni 2011 for the update, Peng et al. 2018 for the energy safeguard)."""
import numpy as np
import pytest

from paper_2203_02054_amd import meshgen as mg
import oracle
from oracle import solver as so


def test_anderson_update_solves_an_affine_fixed_point_in_n_steps():
    """For an affine contraction G(x) = B x + c in R^n, Anderson's type-II
    update with memory n is GMRES on (I - B) x = c in exact arithmetic, so it
    reaches the fixed point (I - B)^-1 c within n + 1 evaluations of G.  A
    wrong sign of the correction, or differences of x where those of G belong,
    does not."""
    rng = np.random.default_rng(3)
    n = 7
    Q = np.linalg.qr(rng.normal(size=(n, n)))[0]
    B = Q @ np.diag(rng.uniform(0.5, 0.99, n)) @ Q.T
    c = rng.normal(size=n)
    x_star = np.linalg.solve(np.eye(n) - B, c)
    x = np.zeros(n)
    xs, fs = [], []
    for _ in range(n + 1):
        g = B @ x + c
        f = g - x
        if xs:
            dX = np.stack([x - xs[-1]] + [xs[i + 1] - xs[i] for i in range(len(xs) - 1)][::-1], axis=1)
            dF = np.stack([f - fs[-1]] + [fs[i + 1] - fs[i] for i in range(len(fs) - 1)][::-1], axis=1)
        else:
            dX = dF = np.zeros((n, 0))
        xs.append(x.copy())
        fs.append(f.copy())
        x, _ = so.anderson_update(g, f, dX, dF)
    assert np.abs(x - x_star).max() < 1e-9 * np.abs(x_star).max()
    # the plain iteration is nowhere near after as many steps
    y = np.zeros(n)
    for _ in range(n + 1):
        y = B @ y + c
    assert np.abs(y - x_star).max() > 1e-2 * np.abs(x_star).max()


def test_anderson_update_without_history_is_the_plain_step():
    g = np.arange(5.0)
    x, gam = so.anderson_update(g, np.ones(5), np.zeros((5, 0)), np.zeros((5, 0)))
    assert np.array_equal(x, g) and gam.size == 0


def _small_block(hyper=True):
    w = mg.block(h=8.0)
    return oracle.Problem.from_workload(w, hyperelastic=hyper, fixed_iters=0), w


@pytest.mark.parametrize("guard", ["residual", "energy", "none"])
def test_accelerated_solve_reaches_the_plain_fixed_point_without_contacts(guard):
    """No collision: the accelerated and plain iterations stop at the same
    fixed point (to the tolerance, amplified by the map's contraction), the
    accelerated one in fewer iterations, whichever guard."""
    prob, w = _small_block()
    xp, _, sp = oracle.solve(prob, w.alpha, tol=1e-11, max_iter=20000)
    xa, _, sa = oracle.solve(prob, w.alpha, tol=1e-11, max_iter=20000, anderson=6, aa_guard=guard)
    assert sp["converged"] and sa["converged"]
    err = np.abs(xa - xp).max() / prob.diag
    print(guard, "plain", sp["iters"], "accelerated", sa["iters"], "rejected", sa["rejected"], "err/diag", err)
    assert err < 1e-8
    assert sa["iters"] < sp["iters"] / 2


def test_residual_guard_rejects_a_growing_residual():
    """The residual guard's rule on a case it must reject: an accelerated
    point whose residual exceeds (1 + slack) times the accepted one's is
    replaced by the plain step from the accepted point (recorded, then
    counted), and never with an infinite slack (a finger with self-contacts,
    where the accelerated residuals do not decrease monotonically)."""
    w = mg.finger(4.0, 4, 2.0)
    prob = oracle.Problem.from_workload(w)
    _, _, s0 = oracle.solve(prob, w.alpha, tol=1e-9, max_iter=2000, anderson=6, aa_guard="residual",
                            aa_slack=0.0, aa_keep_set=False, history=True)
    _, _, s1 = oracle.solve(prob, w.alpha, tol=1e-9, max_iter=2000, anderson=6, aa_guard="residual",
                            aa_slack=np.inf, aa_keep_set=False, history=True)
    H = s0["history"]
    rej = [i for i, h in enumerate(H) if not h["accepted"]]
    assert s0["rejected"] == len(rej) > 0 and s1["rejected"] == 0
    for i in rej:
        acc = [h for h in H[:i] if h["accepted"]][-1]
        assert H[i]["cand"] and H[i]["r"] > acc["r"]


def test_accepted_energies_never_increase_with_an_exact_safeguard():
    """As-rigid-as-possible body targets, no contacts: every plain step lowers
    Eq. 9 (block minimisation); the safeguard (no slack) rejects any
    accelerated point that would not, so the energies of accepted points
    never increase."""
    prob, w = _small_block(hyper=False)
    _, _, sa = oracle.solve(prob, w.alpha, tol=1e-11, max_iter=20000, anderson=6, history=True,
                            aa_guard="energy", aa_slack=0.0)
    E = np.array([h["E"] for h in sa["history"] if h["accepted"]])
    assert sa["converged"] and E.size > 3
    assert np.all(np.diff(E) <= 1e-12 * E[0])


def test_accelerated_solve_with_contacts_stops_at_a_plain_fixed_point():
    """With self-collision and obstacles the set of fixed points depends on
    the path (hysteresis), so the accelerated result is checked as a fixed
    point of the plain map for its own active set: the collision check there
    returns the same set, and a plain step moves it by less than the stopping
    tolerance."""
    from tests.meshes import pressed_finger
    w = pressed_finger()
    prob = oracle.Problem.from_workload(w)
    tol = 1e-9
    xa, A, sa = oracle.solve(prob, w.alpha, tol=tol, max_iter=5000, anderson=8)
    assert sa["converged"] and A.count > 0
    xn, A2, _, info = so.step(prob, xa, w.alpha, A)
    print("accelerated", sa["iters"], "rejected", sa["rejected"], "contacts", A.count, "step", info["r"])
    assert not info["changed"] and info["r"] <= tol


def test_set_guard_lets_only_plain_steps_change_the_active_set():
    """With the set guard, an accelerated point that changed the active set
    is never accepted, and after a rejection the plain step starts from the
    accepted point's set (the plain iteration's state): every change of the
    set is found at a plain point."""
    w = mg.finger(4.0, 4, 2.0)
    prob = oracle.Problem.from_workload(w)
    x, A, st = oracle.solve(prob, w.alpha, tol=1e-9, max_iter=2000, anderson=6, aa_slack=np.inf,
                            aa_keep_set=True, history=True)
    H = st["history"]
    assert st["converged"]
    assert not any(h["cand"] and h["accepted"] and h["changed"] for h in H)
    rej = [h for h in H if not h["accepted"]]
    assert st["rejected"] == len(rej) and all(h["cand"] and h["changed"] for h in rej)
    print("set guard:", st["iters"], "iterations,", st["rejected"], "rejected")


def test_newton_correction_reaches_the_frozen_fixed_point():
    """Newton steps from a point near a frozen-set fixed point converge to it
    quadratically: from a point 4e-4 of the diagonal away, three steps land
    within 1e-10 of the fixed point that the accelerated frozen-set
    iteration finds, each step's map residual roughly the square of the one
    before (relative to the diagonal)."""
    from tests.meshes import pressed_finger
    from oracle import adjoint as oa
    w = pressed_finger()
    prob = oracle.Problem.from_workload(w)
    x, A, st = oracle.solve(prob, w.alpha, fixed_iters=80)
    _, info = oracle.collide(prob, x, A)
    fresh = info["self_fresh"]
    xs, its, step = oa.frozen_solve(prob, w.alpha, x, A, fresh, tol=1e-13)
    rng = np.random.default_rng(1)
    xc = xs + 1e-4 * prob.diag * rng.standard_normal(xs.shape)
    xc[:, prob.fixed] = prob.X0[:, prob.fixed]
    fz = oa._Frozen(prob, A)
    steps = []
    for _ in range(3):
        d, inf = oa.newton_correction(prob, w.alpha, xc, A, fresh, rtol=1e-6, maxiter=300, fz=fz)
        steps.append(inf["step"])
        xc = xc + d
    err = np.abs(xc - xs).max() / prob.diag
    print("newton: map residuals", steps, "distance after three steps", err)
    assert steps[0] > 1e-4 and steps[1] < 1e-5 and steps[2] < 1e-9
    assert err < 1e-10
