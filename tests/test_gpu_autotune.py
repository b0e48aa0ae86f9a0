"""The CG-grid autotuner (gs_autotune): it leaves the caller's positions and
the stored contact set as they were, and the solve it tunes gives the same
result (up to the reduction order of the dot products) with the chosen grid."""
import sys

import numpy as np
import pytest

from paper_2203_02054_amd import meshgen as mg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2203_02054_amd import geosim
    geosim.lib()
    return geosim


def test_autotune_keeps_state_and_result(G):
    w = mg.finger(4.0, 3, 2.0)
    gp = G.Problem.from_workload(w, precision=8, fixed_iters=30, pcg_eta=1e-12, pcg_max=5000, aa_m=0)
    x1, st1 = gp.solve(w.alpha)
    c1 = gp.contacts()
    default_grid = gp.info["pcg_grid"]
    x = x1.clone()
    grid, ms = gp.autotune(w.alpha, x, iters=5)
    print("autotune: default grid", default_grid, "chosen", grid, "ms/iter", ms, flush=True)
    sys.stdout.flush()
    assert grid >= 1 and ms > 0 and gp.info["pcg_grid"] == grid
    assert bool((x == x1).all())                       # positions restored
    c2 = gp.contacts()
    np.testing.assert_array_equal(c1["rows"], c2["rows"])
    np.testing.assert_array_equal(c1["target"], c2["target"])
    gp.reset_contacts()
    x2, st2 = gp.solve(w.alpha)
    diag = gp.info["bbox_diag"]
    err = float((x2 - x1).abs().max()) / diag
    print("  same solve with the chosen grid: err/diag", err, flush=True)
    assert st2["iters"] == st1["iters"] and err < 1e-11
