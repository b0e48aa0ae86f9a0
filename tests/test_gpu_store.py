"""The CG state stored write-back (pcg_store = 2) instead of written through
(pcg_store = 1): only where the bytes travel changes, so every result is the
same bit for bit, with the whole-grid kernel on one mesh and on a batch, in
FP32 and FP64, forward and adjoint."""
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("prec", [4, 8])
def test_write_back_state_gives_the_same_solve_and_gradient(G, prec):
    w = mg.finger(4.0, 3, 2.2)
    verts = np.arange(0, w.n_verts, 7)
    out = {}
    for store in (1, 2):
        # 4 workgroups: more rows per workgroup than lane pairs, so the
        # unpaired whole-grid kernel runs (the one with the write-back variant)
        with G.Problem.from_workload(w, precision=prec, self_collision=1, pcg_blocks=2, pcg_store=store) as gp:
            x, st = gp.solve(w.alpha)
            g = np.zeros((3, w.n_verts))
            g[:, verts] = 1.0
            ga, sa = gp.adjoint(gp.tensor(g))
            out[store] = (x.cpu().numpy(), dict(st), ga.cpu().numpy(), dict(sa))
        say("store", store, out[store][1], out[store][3])
    np.testing.assert_array_equal(out[1][0], out[2][0])
    np.testing.assert_array_equal(out[1][2], out[2][2])
    for k in ("iters", "pcg_iters_total", "status"):
        assert out[1][1][k] == out[2][1][k]
        assert out[1][3][k] == out[2][3][k]


def test_write_back_state_on_a_batch(G):
    wls = [mg.finger(4.0, 3, 2.2), mg.finger(3.0, 4, 1.6), mg.block()]
    alpha = np.concatenate([w.alpha for w in wls])
    res = {}
    for store in (1, 2):
        with G.Problem.batch(wls, precision=4, self_collision=1, pcg_blocks=4, pcg_store=store) as gb:
            x, st = gb.solve(alpha)
            res[store] = (x.cpu().numpy(), dict(st), gb.mesh_iters())
        say("batch store", store, res[store][1], res[store][2])
    np.testing.assert_array_equal(res[1][0], res[2][0])
    np.testing.assert_array_equal(res[1][2], res[2][2])
    assert res[1][1]["pcg_iters_total"] == res[2][1]["pcg_iters_total"]
