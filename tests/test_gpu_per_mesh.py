"""A batch whose global-step CG runs per mesh (pcg_per_mesh = 1).

Each mesh gets its own CG workgroups (the plan gs_cg_plan reports), which
take the step lengths and the stopping test from the mesh's own dot products
(the global step of Section II-C is a separate linear system per mesh) and
wait at barriers for each other only.  A mesh then follows the same path
through the local/global iteration as when it is solved alone with as many CG
workgroups: the same outer iterations, the same CG iterations and the same
positions, bit for bit.  The shared-scalar batch CG (the default) does not
have this property; its iteration counts are only bounded against the
single-mesh ones.
"""
import sys

import numpy as np
import pytest

from paper_2203_02054_amd import meshgen as mg
import oracle

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


def _workloads():
    # uneven sizes and actuations; finger(4, 5, 2.0) settles alone but cycles
    # in a shared-scalar batch with these meshes
    return [mg.finger(4.0, 3, 2.2), mg.finger(3.0, 4, 1.6), mg.finger(4.0, 5, 2.0),
            mg.finger(4.0, 4, np.array([1.2, 2.4, 1.0, 2.0])), mg.block()]


def _split(x, lay, m):
    return x[:, lay["vert"][m]:lay["vert"][m + 1]]


def _each_mesh_alone(G, prec, aa_m, budget, mode):
    wls = _workloads()
    kw = dict(self_collision=1, tol=1e-6 if prec == 4 else 1e-9, aa_m=aa_m, max_iter=4000)
    say("per-mesh batch", prec, aa_m, budget, mode, [w.n_tets for w in wls])
    with G.Problem.batch(wls, precision=prec, pcg_per_mesh=mode, pcg_blocks=budget, **kw) as gp:
        plan = gp.cg_plan()
        alpha = np.concatenate([w.alpha for w in wls])
        xg, st = gp.solve(alpha)
        its = gp.mesh_iters()
        lay = gp.layout()
        xg = xg.cpu().numpy()
    say("  batch:", st, "per-mesh iterations", its, "plan", plan)
    rows = np.diff(lay["vert"])
    assert np.all(plan <= np.maximum(1, rows // 512))
    if mode == 1 and budget == len(wls):
        assert np.all(plan == 1)
    elif mode == 1 or budget == 0:
        assert plan.max() > 1
    assert st["status"] in (G.OK, G.NOT_CONVERGED)
    cg_total = 0
    for m, w in enumerate(wls):
        with G.Problem.from_workload(w, precision=prec, pcg_blocks=int(plan[m]), fixed_iters=0, **kw) as g1:
            assert g1.info["pcg_grid"] == plan[m]
            x1, s1 = g1.solve(w.alpha)
            x1 = x1.cpu().numpy()
        say("  mesh", m, "batch iterations", its[m], "alone", s1["iters"], "CG", s1["pcg_iters_total"],
            "status", s1["status"])
        cg_total += s1["pcg_iters_total"]
        if s1["status"] == G.OK:
            assert its[m] == s1["iters"]
        else:
            assert its[m] == 0  # not converged in either
        np.testing.assert_array_equal(_split(xg, lay, m), x1)
    assert st["pcg_iters_total"] == cg_total


@pytest.mark.parametrize("prec,aa_m,budget", [(4, 8, 0), (4, 0, 0), (8, 8, 0), (4, 8, 5)])
def test_per_mesh_batch_is_each_mesh_alone(G, prec, aa_m, budget):
    """budget 0: the default plan (several workgroups for the larger meshes,
    per-mesh barriers); 5: one workgroup per mesh (block barriers)."""
    _each_mesh_alone(G, prec, aa_m, budget, 1)


@pytest.mark.parametrize("prec,budget", [(4, 0), (8, 0), (4, 3)])
def test_lpt_plan_batch_is_each_mesh_alone(G, prec, budget):
    """The longest-processing-time plan (pcg_per_mesh = 2): the split meshes
    first in block order, the others after them largest first; each mesh is
    still bit for bit its solve alone with as many CG workgroups."""
    _each_mesh_alone(G, prec, 8, budget, 2)


def test_per_mesh_batch_fp64_matches_oracle(G):
    """Fixed iterations with tight CG solves: the per-mesh kernel's positions
    against the FP64 oracle run on each mesh alone."""
    wls = _workloads()[:4]
    K = 25
    with G.Problem.batch(wls, precision=8, self_collision=1, fixed_iters=K, pcg_eta=1e-13, pcg_max=5000,
                         aa_m=0, pcg_per_mesh=1) as gp:
        assert gp.cg_plan().max() > 1
        alpha = np.concatenate([w.alpha for w in wls])
        xg, st = gp.solve(alpha)
        xg = xg.cpu().numpy()
        lay = gp.layout()
    say("per-mesh batch fp64 fixed", st)
    for m, w in enumerate(wls):
        prob = oracle.Problem.from_workload(w)
        xo, _, _ = oracle.solve(prob, w.alpha, fixed_iters=K)
        err = np.abs(_split(xg, lay, m) - xo).max() / prob.diag
        say("  mesh", m, "err/diag", err)
        assert err < 1e-9


def test_per_mesh_frozen_and_single_mesh(G):
    """A batch of one mesh ignores the switch (the whole-grid kernel runs);
    a batch of two copies of a mesh gives each the single-mesh result."""
    w = mg.finger(4.0, 3, 2.0)
    kw = dict(self_collision=1, tol=1e-6, pcg_blocks=1)
    with G.Problem.from_workload(w, precision=4, **kw) as g1:
        x1, s1 = g1.solve(w.alpha)
        x1 = x1.cpu().numpy()
    with G.Problem.batch([w], precision=4, pcg_per_mesh=1, **kw) as gb:
        xb, sb = gb.solve(w.alpha)
        xb = xb.cpu().numpy()
    assert sb["iters"] == s1["iters"]
    np.testing.assert_array_equal(xb, x1)
    with G.Problem.batch([w, w], precision=4, pcg_per_mesh=1, **kw) as g2:
        x2, s2 = g2.solve(np.concatenate([w.alpha, w.alpha]))
        lay = g2.layout()
        x2 = x2.cpu().numpy()
        its = g2.mesh_iters()
    say("two copies", s2, its, "alone", s1)
    assert list(its) == [s1["iters"], s1["iters"]]
    assert s2["pcg_iters_total"] == 2 * s1["pcg_iters_total"]
    for m in range(2):
        np.testing.assert_array_equal(_split(x2, lay, m), x1)


@pytest.mark.parametrize("mode", [1, 2])
def test_per_mesh_adjoint_is_each_mesh_alone(G, mode):
    """The implicit adjoint of a per-mesh batch (plain adjoint iteration, so
    each mesh stops on its own test) gives each mesh the gradient of its
    solve alone, bit for bit, with either workgroup plan."""
    wls = _workloads()[:3]
    kw = dict(self_collision=1, tol=1e-6, adj_aa_m=0, adj_tol=1e-5, adj_max_iter=3000)
    with G.Problem.batch(wls, precision=4, pcg_per_mesh=mode, **kw) as gp:
        plan = gp.cg_plan()
        alpha = np.concatenate([w.alpha for w in wls])
        x, st = gp.solve(alpha)
        lay = gp.layout()
        g = np.zeros((3, gp.n))
        g[:, ::5] = 1.0
        ga, sa = gp.adjoint(gp.tensor(g))
        ga = ga.cpu().numpy()
    say("per-mesh adjoint", sa, "plan", plan)
    c0 = 0
    for m, w in enumerate(wls):
        with G.Problem.from_workload(w, precision=4, pcg_blocks=int(plan[m]), fixed_iters=0, **kw) as g1:
            _, s1 = g1.solve(w.alpha)
            v0, v1 = lay["vert"][m], lay["vert"][m + 1]
            ga1, sa1 = g1.adjoint(g1.tensor(g[:, v0:v1]))
            ga1 = ga1.cpu().numpy()
        say("  mesh", m, "alone adjoint", sa1)
        np.testing.assert_array_equal(ga[c0:c0 + w.n_chambers], ga1)
        c0 += w.n_chambers
