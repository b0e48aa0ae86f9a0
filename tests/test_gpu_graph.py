"""Outer iterations replayed from a captured HIP graph (params.graph = 1).

The graph holds one chunk of check_every outer iterations (every kernel of
the iteration, ordinary launches only, no memory-set nodes); solves with it
must give the eager result bit for bit: positions, iteration counts and
statistics, for every replay, with eager work and synchronisations between
the replays.
"""
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


def _solve_both(G, make, alpha, reps=3):
    import torch
    out = {}
    for graph in (0, 1):
        with make(graph) as gp:
            res = []
            for r in range(reps):
                gp.reset_contacts()
                x, st = gp.solve(alpha)
                torch.cuda.synchronize()
                # eager work on the device between the replays
                y = (x * 2.0).sum().item()
                res.append((x.cpu().numpy(), dict(st), y))
            out[graph] = res
    return out


def _check(out, say_tag):
    x0, st0, _ = out[0][0]
    for graph in (0, 1):
        for r, (x, st, _) in enumerate(out[graph]):
            say(say_tag, "graph", graph, "rep", r, st["iters"], st["pcg_iters_total"], st["status"])
            np.testing.assert_array_equal(x, x0)
            for k in ("iters", "pcg_iters_total", "n_contacts", "status", "aa_rejected"):
                assert st[k] == st0[k], (graph, r, k)
            assert st["residual"] == st0["residual"]


@pytest.mark.parametrize("prec", [4, 8])
def test_graph_solve_equals_eager_finger(G, prec):
    w = mg.finger(4.0, 3, 2.2)
    tol = 1e-6 if prec == 4 else 1e-9
    out = _solve_both(G, lambda g: G.Problem.from_workload(w, precision=prec, self_collision=1, tol=tol,
                                                           check_every=8, graph=g), w.alpha)
    assert out[1][0][1]["iters"] > 16  # several chunks came from the graph
    _check(out, f"finger fp{8 * prec}")


def test_graph_solve_equals_eager_per_mesh_batch(G):
    wls = [mg.finger(4.0, 3, 2.2), mg.finger(3.0, 4, 1.6), mg.block()]
    alpha = np.concatenate([w.alpha for w in wls])
    out = _solve_both(G, lambda g: G.Problem.batch(wls, precision=4, self_collision=1, pcg_per_mesh=1,
                                                   check_every=16, graph=g), alpha)
    _check(out, "per-mesh batch")


def test_graph_follows_changed_parameters(G):
    """A parameter change gives new kernel arguments: the graph is captured
    again and the result is the eager one for the new parameters."""
    w = mg.finger(3.0, 4, 1.6)
    with G.Problem.from_workload(w, precision=4, self_collision=1, check_every=8, graph=1) as gp, \
            G.Problem.from_workload(w, precision=4, self_collision=1, check_every=8, graph=0) as ge:
        for tol in (1e-5, 1e-6):
            gp.set_params(tol=tol)
            ge.set_params(tol=tol)
            gp.reset_contacts()
            ge.reset_contacts()
            xg, sg = gp.solve(w.alpha)
            xe, se = ge.solve(w.alpha)
            say("tol", tol, sg["iters"], se["iters"])
            assert sg["iters"] == se["iters"]
            np.testing.assert_array_equal(xg.cpu().numpy(), xe.cpu().numpy())
