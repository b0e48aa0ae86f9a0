"""The refit-only AABB tree over the tets (the paper's broadphase, Section
II-B) against the spatial hash the solver uses and the oracle's brute force:
at every tested state the three candidate sets C_tet are identical, pair for
pair (the set is fixed by its definition; any correct broadphase returns it).
"""
import sys

import numpy as np
import pytest

from paper_2203_02054_amd import meshgen as mg
import oracle
from oracle.collision import tet_candidates
from tests.meshes import pressed_finger, wavy_positions

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


def _oracle_pairs(prob, x, broadphase="brute"):
    v, e, _ = tet_candidates(prob, x, prob.query_verts, broadphase=broadphase)
    pr = np.stack([v, e], axis=1).astype(np.int64)
    return pr[np.lexsort((pr[:, 1], pr[:, 0]))]


@pytest.mark.parametrize("precision", [8, 4])
def test_tree_hash_and_brute_force_agree_on_the_finger(G, precision):
    w = pressed_finger()
    prob = oracle.Problem.from_workload(w)
    x1, _, _ = oracle.solve(prob, w.alpha, fixed_iters=20)
    rng = np.random.default_rng(41)
    states = [prob.X0, x1, wavy_positions(prob.X0, rng, 0.8 * prob.h_ref, noise=0.2 * prob.h_ref)]
    dt = np.float64 if precision == 8 else np.float32
    with G.Problem.from_workload(w, precision=precision) as gp:
        for i, x in enumerate(states):
            x = x.astype(dt).astype(np.float64)
            xt = gp.tensor(x)
            tree, t_refit, t_query = gp.tree_candidates(xt)
            hashed = gp.collide(xt)["cand_tet"]
            brute = _oracle_pairs(prob, x)
            say(f"state {i}: {tree.shape[0]} candidate pairs; tree refit {t_refit:.3f} ms, query {t_query:.3f} ms")
            np.testing.assert_array_equal(tree, brute)
            np.testing.assert_array_equal(hashed, brute)
            if i > 0:
                assert tree.shape[0] > 0


def test_tree_and_hash_agree_on_the_gripper(G):
    w = mg.gripper()
    prob = oracle.Problem.from_workload(w)
    rng = np.random.default_rng(42)
    x = wavy_positions(prob.X0, rng, 0.6 * prob.h_ref, noise=0.1 * prob.h_ref).astype(np.float32)
    with G.Problem.from_workload(w, precision=4) as gp:
        xt = gp.tensor(x)
        tree, t_refit, t_query = gp.tree_candidates(xt)
        tree, t_refit, t_query = gp.tree_candidates(xt)        # timed after the first (topology) call
        hashed = gp.collide(xt)["cand_tet"]
        say(f"gripper: {tree.shape[0]} pairs; tree refit {t_refit:.3f} ms, query {t_query:.3f} ms")
        np.testing.assert_array_equal(tree, hashed)
        kd = _oracle_pairs(prob, x.astype(np.float64), broadphase="kdtree")
        np.testing.assert_array_equal(tree, kd)
        assert tree.shape[0] > 1000
