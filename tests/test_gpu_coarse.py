"""The CG kernel's coarse correction (a two-level preconditioner: Jacobi plus
one coarse unknown per workgroup's row range, A0 = R0 A_el R0^T) against the
oracle.  A preconditioner changes how the global step's CG reaches its
tolerance, not the solution, so with exact inner solves the FP64 iteration
must follow the oracle's (sparse direct global steps) as the Jacobi-only
kernel does; on the gripper the coarse correction must also take far fewer
CG iterations.
"""
import sys

import numpy as np
import pytest

from paper_2203_02054_amd import meshgen as mg
import oracle
from tests.meshes import pressed_finger

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


def test_fp64_iteration_with_the_coarse_correction_follows_the_oracle(G):
    w = pressed_finger()
    K = 30
    prob = oracle.Problem.from_workload(w)
    xo, Ao, _ = oracle.solve(prob, w.alpha, fixed_iters=K)
    orows, _ = Ao.listing(prob)
    its = {}
    for cz in (0, 1):
        with G.Problem.from_workload(w, precision=8, fixed_iters=K, aa_m=0, pcg_eta=1e-12, pcg_max=5000,
                                     pcg_coarse=cz) as gp:
            xg, st = gp.solve(w.alpha)
            err = np.abs(xg.cpu().numpy() - xo).max() / prob.diag
            say("coarse", cz, "grid", gp.info["pcg_grid"], st, "err/diag", err)
            assert gp.info["pcg_grid"] >= 2
            np.testing.assert_array_equal(gp.contacts()["rows"], orows)
            assert err < 1e-9
            its[cz] = st["pcg_iters_total"]
    # three row ranges are too few coarse unknowns to cut this small mesh's
    # CG work (the gripper test below measures the cut)
    say("CG iterations", its)


@pytest.mark.parametrize("precision", [8, 4])
def test_adjoint_with_the_coarse_correction_matches_the_plain_one(G, precision):
    """The implicit adjoint's CG uses the same kernel: with and without the
    coarse correction the gradients agree (FP64 at tolerance 1e-10 to 1e-9;
    FP32 at the default adjoint tolerance 1e-6 to 1e-3, the FP32 gradient bar)."""
    w = pressed_finger()
    rng = np.random.default_rng(8)
    g = rng.normal(size=w.rest_xyz.shape)
    out = {}
    for cz in (0, 1):
        # two workgroups: the unpaired kernel (which carries the coarse
        # correction) in FP32 as well
        tol = dict(pcg_eta=1e-10, adj_tol=1e-10) if precision == 8 else dict(pcg_eta=1e-5, adj_tol=1e-6)
        with G.Problem.from_workload(w, precision=precision, fixed_iters=40, aa_m=0, pcg_max=5000,
                                     pcg_coarse=cz, pcg_blocks=2, **tol) as gp:
            gp.solve(w.alpha)
            ga, st = gp.adjoint(g)
            out[cz] = (ga.cpu().numpy().astype(np.float64), st)
            say("adjoint coarse", cz, st)
    rel = np.linalg.norm(out[1][0] - out[0][0]) / np.linalg.norm(out[0][0])
    say("relative difference", rel)
    assert rel < (1e-9 if precision == 8 else 1e-3)


def test_gripper_cg_iterations_drop_with_the_coarse_correction(G):
    """The first 40 outer iterations of the gripper on 128 workgroups: the
    same inner tolerance reached in far fewer CG iterations, and the two
    iterations stay close (their inexact global steps differ)."""
    w = mg.make("gripper")
    res = {}
    for cz in (0, 1):
        with G.Problem.from_workload(w, precision=4, pcg_blocks=128, fixed_iters=40, pcg_coarse=cz) as gp:
            x, st = gp.solve(w.alpha)
            res[cz] = (x.cpu().numpy(), st)
            say("gripper coarse", cz, st)
    ratio = res[1][1]["pcg_iters_total"] / res[0][1]["pcg_iters_total"]
    diff = np.abs(res[1][0] - res[0][0]).max() / np.ptp(w.rest_xyz, axis=1).max()
    say("CG iteration ratio", ratio, "max |dx| over the box size", diff)
    assert ratio < 0.6
    assert diff < 5e-2
