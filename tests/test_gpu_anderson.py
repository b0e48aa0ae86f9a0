"""The Anderson-accelerated local/global iteration on the GPU (the acceleration
the paper applies to its solver, end of Section III-B) against the oracle:

* FP64 kernels with an exact inner solve follow the oracle's accelerated
  iteration at matched iteration counts (residual guard; energy guard on an
  as-rigid-as-possible block), with the same contact sets and rejections;
* the FP32 accelerated solve stops at a fixed point of the oracle's plain
  map for its own active set, in fewer iterations than the plain path;
* a grid barrier that gives up (forced by a zero wait limit) returns an
  error and leaves the problem usable.
"""
import sys

import numpy as np
import pytest

from paper_2203_02054_amd import meshgen as mg
import oracle
from tests import fixed_point as fp

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


def test_fp64_accelerated_iteration_matches_oracle_at_matched_iterations(G):
    w = mg.finger(4.0, 4, 2.0)
    prob = oracle.Problem.from_workload(w)
    K = 60
    gp = G.Problem.from_workload(w, precision=8, pcg_eta=1e-13, pcg_max=5000, fixed_iters=K, aa_m=8,
                                 aa_guard=G.AA_GUARD_RESIDUAL | G.AA_GUARD_SET, aa_slack=0.5)
    xg, st = gp.solve(w.alpha)
    xo, Ao, so = oracle.solve(prob, w.alpha, fixed_iters=K, anderson=8, aa_guard="residual", aa_slack=0.5,
                              aa_keep_set=True)
    err = np.abs(xg.cpu().numpy() - xo).max() / prob.diag
    orows, _ = Ao.listing(prob)
    say("accelerated fp64 finger:", st, "oracle rejected", so["rejected"], "err/diag", err)
    np.testing.assert_array_equal(gp.contacts()["rows"], orows)
    assert st["aa_rejected"] == so["rejected"]
    # the GPU solves the least-squares step through its normal equations with
    # a ridge of 1e-10 of the largest Gram entry, the oracle with numpy's
    # lstsq; the accelerated updates pass the coefficients' differences on
    # (1.8e-8 of the diagonal after 60 iterations, measured)
    assert err < 1e-7


def test_fp64_energy_guard_matches_oracle_on_an_arap_block(G):
    w = mg.block(h=8.0)
    prob = oracle.Problem.from_workload(w, hyperelastic=False, fixed_iters=0)
    K = 40
    gp = G.Problem.from_workload(w, precision=8, hyperelastic=0, pcg_eta=1e-13, pcg_max=5000, fixed_iters=K,
                                 aa_m=6, aa_guard=G.AA_GUARD_ENERGY, aa_slack=0.0)
    xg, st = gp.solve(w.alpha)
    xo, _, so = oracle.solve(prob, w.alpha, fixed_iters=K, anderson=6, aa_guard="energy", aa_slack=0.0,
                             aa_keep_set=False)
    err = np.abs(xg.cpu().numpy() - xo).max() / prob.diag
    say("energy guard fp64 block:", st, "oracle rejected", so["rejected"], "err/diag", err)
    assert st["aa_rejected"] == so["rejected"]
    assert err < 1e-9


def test_fp32_accelerated_solve_stops_at_an_oracle_fixed_point(G):
    w = mg.finger(4.0, 4, 2.0)
    prob = oracle.Problem.from_workload(w)
    gp = G.Problem.from_workload(w, precision=4, tol=1e-7)
    xg, st = gp.solve(w.alpha)
    gq = G.Problem.from_workload(w, precision=4, tol=1e-7, aa_m=0)
    _, sq = gq.solve(w.alpha)
    say("fp32 finger tol 1e-7: accelerated", st, "plain", sq)
    assert st["status"] == G.OK and sq["status"] == G.OK
    assert st["iters"] < sq["iters"]
    r = fp.check(prob, w.alpha, xg.cpu().numpy().astype(np.float64), gp.contacts())
    say("  oracle fixed point for the GPU set:", r["iters"], "iterations, err/diag", r["err"],
        "same set", r["same_set"], "contacts", r["contacts"])
    assert r["same_set"] and r["err"] < 1e-5


def test_batched_accelerated_meshes_keep_their_own_history(G):
    """Two copies of one mesh in a batch with a third, different mesh: each
    copy's accelerated path is the single-mesh path (per-mesh histories,
    decisions and least-squares solves), so their results agree with each
    other to rounding of the shared CG scalars, and every mesh converges."""
    a = mg.finger(4.0, 3, 2.0)
    b = mg.finger(4.0, 4, 1.6)
    gb = G.Problem.batch([a, b, a], precision=8, self_collision=1, tol=1e-8, pcg_eta=1e-12, pcg_max=5000)
    alpha = np.concatenate([a.alpha, b.alpha, a.alpha])
    xg, st = gb.solve(alpha)
    its = gb.mesh_iters()
    lay = gb.layout()
    x = xg.cpu().numpy()
    x0 = x[:, lay["vert"][0]:lay["vert"][1]]
    x2 = x[:, lay["vert"][2]:lay["vert"][3]]
    say("batched accelerated:", st, "per-mesh iterations", its, "copy difference", np.abs(x0 - x2).max())
    assert st["status"] == G.OK and np.all(its > 0)
    assert np.abs(x0 - x2).max() < 1e-9 * np.abs(x0).max()


def test_barrier_give_up_returns_an_error_and_the_problem_stays_usable(G):
    """With a zero wait limit every grid barrier gives up at its first
    unfinished poll: the CG kernel's workgroups all leave, the solve returns
    GS_EHIP with the barrier's message, and after restoring the limit the
    same problem solves to the result of a fresh one."""
    w = mg.finger(4.0, 4, 2.0)
    gp = G.Problem.from_workload(w, precision=4, barrier_timeout_ms=0.0)
    assert gp.info["pcg_grid"] >= 2
    with pytest.raises(G.GeosimError) as ei:
        gp.solve(w.alpha)
    say("forced give-up:", ei.value)
    assert ei.value.code == G.EHIP and "barrier" in str(ei.value)
    gp.set_params(barrier_timeout_ms=2000.0)
    gp.reset_contacts()
    x1, s1 = gp.solve(w.alpha)
    g2 = G.Problem.from_workload(w, precision=4)
    x2, s2 = g2.solve(w.alpha)
    say("  after restoring the limit:", s1, s2)
    assert s1 == s2 and bool((x1 == x2).all())
