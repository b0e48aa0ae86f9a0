"""The allocation-free collision check (gs_collide_debug_static, candidate
lists staged in the library's static device array) against gs_collide_debug
with a caller-provided scratch, through the C ABI: two calls in a row, the
second on a smaller mesh with a smaller capacity, each bit for bit equal to
the scratch entry point's result (candidate pairs, contact rows, targets)."""
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


def _state(G, w, iters):
    gp = G.Problem.from_workload(w, precision=4, fixed_iters=iters, aa_m=0)
    x, st = gp.solve(w.alpha)
    return gp, x, st


def test_static_collision_check_matches_the_scratch_entry_point(G):
    cases = [(mg.finger(4.0, 4, 2.0), 60, 60000), (mg.finger(4.0, 2, 2.0), 25, 20000)]
    sizes = []
    for w, iters, cap in cases:
        gp, x, st = _state(G, w, iters)
        a = gp.collide_static(x, cap=cap)
        b = gp.collide(x, cap=cap)
        print(w.n_tets, "tets:", {k: v.shape for k, v in a.items()}, flush=True)
        sys.stdout.flush()
        for k in ("cand_tet", "cand_tri", "contacts", "target"):
            np.testing.assert_array_equal(a[k], b[k])
        assert a["cand_tet"].shape[0] > 0 and a["contacts"].shape[0] > 0
        sizes.append((w.n_tets, a["cand_tet"].shape[0]))
        gp.close()
    assert sizes[1][0] < sizes[0][0]


def test_static_collision_check_refuses_a_capacity_beyond_its_array(G):
    w = mg.finger(4.0, 3, 2.0)
    gp, x, _ = _state(G, w, 2)
    with pytest.raises(G.GeosimError) as ei:
        gp.collide_static(x, cap=G.STATIC_CAND_CAP + 1)
    assert ei.value.code == G.EINVAL and "static" in str(ei.value)
    gp.close()
