"""Parity at full size: the three-finger gripper (378,666 tets) and the
256-mesh batch (5.56M tets), in the FP32 configuration the benchmark runs,
on outputs the oracle can compute at that size:

* gripper, after 30 GPU iterations from rest (a deformed state with self,
  sphere and plane contacts):
  - the local step on every tet against the oracle's;
  - tet candidates, penetration and ray hits of a sample of query vertices
    against the oracle's brute force restricted to that sample (bit-exact);
  - one FP64 global step with the GPU's contact set against the oracle's
    sparse direct solve;
* gripper gradient workload (30 fingertip targets, 24 chamber ratios):
  unrolled adjoint over 20 iterations, FP64 and FP32 kernels, against FP64
  central differences of the 20-iteration solve;
* batch: every sampled converged mesh is a fixed point of the oracle's
  iteration with its own active set (one oracle step leaves the set
  unchanged and moves it by less than 5e-6 of its diagonal).
"""
import sys

import numpy as np
import pytest

from paper_2203_02054_amd import meshgen as mg
import oracle
from oracle import collision as oc
from oracle import solver as osolver
from oracle.collision import Contacts

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2203_02054_amd import geosim
    geosim.lib()
    return geosim


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle_contacts(prob, cg, lo=0):
    A = Contacts.empty(prob.query_verts.size, prob.n_slots)
    ns = prob.spheres.shape[0]
    for (v, typ, prim), t, nrm in zip(cg["rows"], cg["target"], cg["normal"]):
        s = int(np.searchsorted(prob.query_verts, v - lo))
        sl = 0 if typ == 0 else (1 + prim if typ == 1 else 1 + ns + prim)
        A.active[s, sl] = True
        A.target[s, sl], A.normal[s, sl], A.prim[s, sl] = t, nrm, prim
    return A


@pytest.fixture(scope="module")
def gripper_state(G):
    w = mg.gripper()
    prob = oracle.Problem.from_workload(w)
    gp = G.Problem.from_workload(w, precision=4, fixed_iters=30)
    x, st = gp.solve(w.alpha)
    say("gripper", w.n_tets, "tets: 30 iterations", st)
    return w, prob, gp, x


def test_gripper_local_step_full(G, gripper_state):
    w, prob, gp, x = gripper_state
    xs = x.cpu().numpy().astype(np.float64)
    Tg = gp.local_step(x, w.alpha).cpu().numpy().astype(np.float64)       # [3, 4, T]
    To = oracle.local_step(prob, xs, w.alpha)                              # [T, 3, 4]
    err = np.abs(np.moveaxis(Tg, 2, 0) - To).max() / prob.diag
    say("  local step on", prob.T, "tets: max error / diag", err)
    assert err < 1e-5


def test_gripper_collision_sampled(G, gripper_state):
    w, prob, gp, x = gripper_state
    x32 = x.cpu().numpy()
    x64 = x32.astype(np.float64)
    got = gp.collide(x)
    # every 97th query vertex plus every vertex with a contact at this state
    sample = np.union1d(prob.query_verts[::97], got["contacts"][:, 0]).astype(np.int64)
    v, e, inside = oc.tet_candidates(prob, x64, sample)
    exp = np.unique(np.stack([v, e], axis=1), axis=0)
    gt = got["cand_tet"]
    mine = gt[np.isin(gt[:, 0], sample)]
    say("  sampled", sample.size, "query vertices: tet candidates", len(exp), "penetrating",
        np.unique(v[inside]).size, "contacts", len(got["contacts"]))
    np.testing.assert_array_equal(mine, exp)
    # rays of the sampled penetrating vertices
    pen = np.unique(v[inside])
    if pen.size:
        nrm, ok = oc.vertex_normals(prob, x64, pen)
        hit, bf, bt, cand = oc.ray_cast(prob, x64, pen[ok], nrm[:, ok])
        ctri = got["cand_tri"]
        ctri = ctri[np.isin(ctri[:, 0], pen[ok])]
        exp_tri = np.unique(np.stack(cand, axis=1), axis=0) if cand[0].size else np.zeros((0, 2), np.int64)
        np.testing.assert_array_equal(ctri, exp_tri)
        rows = got["contacts"]
        for vv, h, f in zip(pen[ok], hit, bf):
            r = rows[(rows[:, 0] == vv) & (rows[:, 1] == 0)]
            if h:
                assert len(r) == 1 and r[0, 2] == f


@pytest.mark.parametrize("coarse", [0, 1])
def test_gripper_global_step_fp64(G, gripper_state, coarse):
    """One FP64 iteration from the FP32 state with the GPU's contacts, against
    the oracle's local step plus sparse direct global step with the contact
    set the GPU found in that iteration; with and without the CG's coarse
    correction (on 128 workgroups)."""
    w, prob, _, x = gripper_state
    kw = dict(pcg_coarse=1, pcg_blocks=128) if coarse else {}
    gp = G.Problem.from_workload(w, precision=8, fixed_iters=1, pcg_eta=1e-13, pcg_max=20000, **kw)
    x0 = x.double().contiguous()
    x1, st = gp.solve(w.alpha, x0.clone())
    # the solve holds fixed vertices at their rest positions (not at their
    # FP32 roundings): the oracle starts from the same positions
    xs = x0.cpu().numpy()
    xs[:, prob.fixed] = prob.X0[:, prob.fixed]
    cg = gp.contacts()
    A = _oracle_contacts(prob, cg)
    Tt = oracle.local_step(prob, xs, w.alpha)
    xo = osolver.global_step(prob, Tt, A, xs)
    xg = x1.cpu().numpy()
    err = np.abs(xg - xo).max() / prob.diag
    # the GPU's global step is a CG stopped at a 1e-13 relative residual; its
    # residual in the oracle's system is the solver-independent check, the
    # position error carries the condition number of M (long fingers)
    M, _, bs = osolver.system(prob, A)
    F, C = np.nonzero(prob.free)[0], np.nonzero(prob.fixed)[0]
    b = (osolver.element_rhs(prob, Tt) + bs)[:, F].T - M[F][:, C] @ xs[:, C].T
    res = np.linalg.norm(M[F][:, F] @ xg[:, F].T - b) / np.linalg.norm(b)
    say("  one FP64 iteration:", st, "contacts", len(cg["rows"]), "relative residual", res,
        "max error / diag", err)
    assert res < 1e-11 and err < 1e-8


def test_batch_sampled_meshes_are_oracle_fixed_points(G):
    """The 256-mesh batch (5.56M tets, accelerated): 16 of the meshes that
    converged within the cap, spread over the size range (every 1/16 quantile
    of their tet counts), are fixed points of the oracle's map to the
    tolerance scale with their own contact sets: one oracle step from the GPU
    result moves it by at most 2e-6 of the diagonal and keeps the set.  How
    far such a point lies from the exact fixed point depends on the mesh's
    condition: for the smallest converged mesh (4,752 tets, a 6.4e-7 step)
    the oracle's frozen-set iteration lands 2.9e-4 of the diagonal away
    (measured), so the distance is not asserted here.  The meshes that did
    not converge are counted (active-set cycles, see the design notes)."""
    wls = mg.batched(256)
    gb = G.Problem.batch(wls, precision=4, self_collision=1, max_iter=1000)
    alpha = np.concatenate([w.alpha for w in wls])
    xg, st = gb.solve(alpha)
    its = gb.mesh_iters()
    conv = np.nonzero(its > 0)[0]
    say("batch", sum(w.n_tets for w in wls), "tets:", st, "converged", conv.size, "not converged",
        int((its == 0).sum()))
    lay = gb.layout()
    cg = gb.contacts()
    xg = xg.cpu().numpy().astype(np.float64)
    Ts = np.array([wls[m].n_tets for m in conv])
    order = conv[np.argsort(Ts, kind="stable")]
    picks = list(dict.fromkeys(order[np.linspace(0, order.size - 1, 16).round().astype(int)].tolist()))
    assert len(picks) >= 12
    for m in picks:   # smallest first
        w = wls[m]
        prob = oracle.Problem.from_workload(w, self_collision=True)
        v0, v1 = lay["vert"][m], lay["vert"][m + 1]
        sel = (cg["rows"][:, 0] >= v0) & (cg["rows"][:, 0] < v1)
        sub = {k: cg[k][sel] for k in ("rows", "target", "normal")}
        A = _oracle_contacts(prob, sub, lo=v0)
        x = xg[:, v0:v1]
        xn, A2, _, info = osolver.step(prob, x, w.alpha, A)
        move = np.abs(xn - x).max() / prob.diag
        say("  mesh", m, w.n_tets, "tets, converged at", its[m], ": oracle step moves", move,
            "set changed", info["changed"])
        assert not info["changed"] and move < 2e-6


def test_gripper_unrolled_gradient_vs_central_differences(G):
    """The gradient workload at full size: loss = squared distance of 30
    fingertip vertices to seeded targets, gradient w.r.t. the 24 chamber
    volume ratios through 20 iterations from rest.  FP32 and FP64 unrolled
    adjoints against FP64 central differences (h = 1e-6) of the FP64
    20-iteration solve, whose contact schedule is checked unchanged at
    alpha +- h."""
    import torch
    w = mg.gripper()
    K = 20
    verts, y = mg.adjoint_targets(w)
    tight = dict(pcg_eta=1e-13, pcg_max=20000)
    g64 = G.Problem.from_workload(w, precision=8, fixed_iters=K, aa_m=0, **tight)

    def loss_and_contacts(alpha):
        g64.reset_contacts()
        x, _ = g64.solve(alpha)
        xv = x.cpu().numpy()[:, verts]
        return float(((xv - y.T) ** 2).sum()), g64.contacts()["rows"]

    L0, rows0 = loss_and_contacts(w.alpha)
    g64.reset_contacts()
    xK = g64.solve(w.alpha)[0].cpu().numpy()
    dLdx = np.zeros((3, w.n_verts))
    dLdx[:, verts] = 2.0 * (xK[:, verts] - y.T)
    h = 1e-6
    fd = np.zeros(w.n_chambers)
    for c in range(w.n_chambers):
        ap, am = w.alpha.copy(), w.alpha.copy()
        ap[c] += h
        am[c] -= h
        Lp, rp = loss_and_contacts(ap)
        Lm, rm = loss_and_contacts(am)
        np.testing.assert_array_equal(rp, rows0)
        np.testing.assert_array_equal(rm, rows0)
        fd[c] = (Lp - Lm) / (2 * h)
    out = {}
    for prec, kw in [(8, tight), (4, dict(pcg_eta=1e-6, pcg_max=5000))]:
        gp = G.Problem.from_workload(w, precision=prec, **kw)
        ga, _, _, st = gp.adjoint_unrolled(w.alpha, K, dLdx)
        ga = ga.cpu().numpy().astype(np.float64)
        out[prec] = np.linalg.norm(ga - fd) / np.linalg.norm(fd)
        say("  unrolled", prec, st, "rel to FD", out[prec])
    say("  FD", fd[:6], "...")
    # FP32: the error plateaus at 4e-3 for CG tolerances from 1e-5 to 1e-7 (the
    # rounding floor of FP32 reverse solves with the long fingers' stiffness
    # matrix); the FP64 kernels meet the FD to 3e-6
    assert out[8] < 1e-5 and out[4] < 1e-2


def test_gripper_converged_solve_is_a_fixed_point_of_the_oracle_map(G):
    """The benchmark's gripper solve (FP32, accelerated, tol 1e-6) converges,
    and its result is a fixed point of the oracle's map for its own active
    set to the stopping tolerance: one step of the oracle's frozen-set map
    (exact sparse global step, FP64) moves it by at most 2e-6 of the
    diagonal, and the oracle's collision check there (exact k-d tree
    broadphase, checked equal to brute force) returns the same active set
    with the same fresh/kept targets.  The distance to the exact fixed point
    is not asserted here: at this state the map's fixed-point problem has a
    condition of about 3e4 (a Newton step of 2.6e-2 of the diagonal against
    a map residual of 9.1e-7, measured with the oracle's newton_correction),
    so a 1e-6 residual fixes the positions only to about that, in FP32 or
    FP64 alike."""
    from oracle import adjoint as oa
    from tests import fixed_point as fp
    w = mg.gripper()
    prob = oracle.Problem.from_workload(w)
    gp = G.Problem.from_workload(w, precision=4)
    x, st = gp.solve(w.alpha)
    say("gripper bench solve:", st)
    assert st["status"] == G.OK and st["residual"] <= 1e-6
    xg = x.cpu().numpy().astype(np.float64)
    cg = gp.contacts()
    A, fresh = fp.oracle_contacts(prob, cg)
    xn = oa.frozen_map(prob, xg, w.alpha, A, fresh)
    step = np.abs(xn - xg).max() / prob.diag
    A2, info = oracle.collide(prob, xg, A, broadphase="kdtree")
    same = (A2.same_set(A) and np.array_equal(A2.prim[A.active], A.prim[A.active])
            and np.array_equal(info["self_fresh"], fresh))
    say("  oracle map step from the GPU result", step, "contacts", A.count, "same set", same)
    assert step <= 2e-6
    assert same
