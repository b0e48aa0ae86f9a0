"""Edge cases of the GPU path through the C ABI, each checked against the FP64
oracle or a closed form:

* every CG kernel variant and both launch kinds. FP32 solves follow the
  oracle's trajectory to the matched-iteration bar (1e-5 of the diagonal,
  contact rows equal) in three configurations:
  - one block (more than 256 rows: the unpaired kernel, ordinary launch);
  - the default grid (the paired-lane kernel, ordinary launch);
  - the largest resident grid (paired-lane kernel, cooperative launch);
* obstacle contacts without self-collision. The local step runs as its own
  launch and the contact update rides in the gather. FP64 against the oracle
  at matched iterations (1e-9 of the diagonal, contact rows equal);
* a single tet, where every array is ragged (4 vertices, 1 tet, 1 block). One
  chamber with one fixed vertex reaches the closed-form fixed point
  x = x_f + alpha^(1/3) (X - x_f) (Eq. 6 with R = I) in FP64 and FP32;
* a mesh whose vertices are all fixed. There are no query vertices and no
  free rows: the solve returns the rest shape at once, and the gradient
  with respect to its chamber is zero;
* a mesh without chambers: the solve and the adjoint run with an empty
  actuation vector;
* the FP32 implicit and unrolled adjoints in both CG state layouts. One
  block runs the unpaired kernel (rows of three vectors); the default grid
  runs the paired kernel (three arrays of rows). The gradients agree.
"""
import dataclasses
import sys

import numpy as np
import pytest

from paper_2203_02054_amd import meshgen as mg
import oracle
from tests.meshes import pressed_finger, voxel_box

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


@pytest.fixture(scope="module")
def finger_oracle_150():
    wl = mg.finger(4.0, 4, 2.0)
    prob = oracle.Problem.from_workload(wl)
    xo, Ao, _ = oracle.solve(prob, wl.alpha, fixed_iters=150)
    rows, _ = Ao.listing(prob)
    return wl, prob, xo, rows


@pytest.mark.parametrize("blocks", [1, 0, 1 << 20])
def test_cg_variants_and_launch_kinds_follow_the_oracle(G, finger_oracle_150, blocks):
    wl, prob, xo, orows = finger_oracle_150
    gp = G.Problem.from_workload(wl, precision=4, pcg_eta=1e-7, pcg_max=3000, fixed_iters=150,
                                 pcg_blocks=blocks, aa_m=0)
    grid = gp.info["pcg_grid"]
    rows_per_block = ((gp.n + grid - 1) // grid + 63) // 64 * 64
    say("finger fp32, pcg_blocks", blocks, "-> grid", grid, "rows per block", rows_per_block)
    if blocks == 1:
        assert grid == 1 and rows_per_block > 256
    if blocks == 1 << 20:
        assert grid >= 128 and rows_per_block <= 256
    xg, st = gp.solve(wl.alpha)
    err = np.abs(xg.cpu().numpy().astype(np.float64) - xo).max() / prob.diag
    say("  ", st, "err/diag", err)
    np.testing.assert_array_equal(gp.contacts()["rows"], orows)
    assert err < 1e-5


def test_obstacles_without_self_collision_match_oracle(G):
    w = dataclasses.replace(pressed_finger(), self_collision=False)
    prob = oracle.Problem.from_workload(w)
    K = 40
    gp = G.Problem.from_workload(w, precision=8, pcg_eta=1e-13, pcg_max=5000, fixed_iters=K, aa_m=0)
    xg, st = gp.solve(w.alpha)
    xo, Ao, _ = oracle.solve(prob, w.alpha, fixed_iters=K)
    err = np.abs(xg.cpu().numpy() - xo).max() / prob.diag
    rows = gp.contacts()["rows"]
    orows, _ = Ao.listing(prob)
    say("obstacles only:", st, "contacts", len(rows), "types", np.bincount(rows[:, 1], minlength=3) if len(rows) else [],
        "err/diag", err)
    assert len(rows) > 0 and np.all(rows[:, 1] != 0)
    np.testing.assert_array_equal(rows, orows)
    assert err < 1e-9


@pytest.mark.parametrize("precision", [8, 4])
def test_single_tet_reaches_the_closed_form(G, precision):
    X = np.array([[0.0, 2.0, 0.0, 0.0], [0.0, 0.0, 2.0, 0.0], [0.0, 0.0, 0.0, 2.0]])
    tets = np.array([[0], [1], [2], [3]], np.int32)
    fixed = np.array([1, 0, 0, 0], np.uint8)
    alpha = 1.5
    kw = dict(pcg_eta=1e-13, pcg_max=100) if precision == 8 else {}
    gp = G.Problem(X, tets, np.array([mg.CH_ISO], np.uint8), np.array([0], np.int16), fixed, 1,
                   precision=precision, self_collision=1, fixed_iters=3, **kw)
    xg, st = gp.solve([alpha])
    exact = X[:, :1] + alpha ** (1.0 / 3.0) * (X - X[:, :1])
    err = np.abs(xg.cpu().numpy().astype(np.float64) - exact).max()
    say("single tet", precision, st, "err", err)
    assert st["n_contacts"] == 0
    assert err < (1e-12 if precision == 8 else 2e-6)


@pytest.mark.parametrize("precision", [8, 4])
def test_all_fixed_mesh_returns_rest_shape_with_zero_gradient(G, precision):
    m = voxel_box(2, 1, 1, h=1.0, mode=mg.CH_ISO, chamber=0)
    m["fixed"][:] = 1
    gp = G.Problem(m["rest_xyz"], m["tets"], m["tet_mode"], m["tet_chamber"], m["fixed"], 1,
                   precision=precision, self_collision=1)
    assert gp.info["n_query_verts"] == 0
    xg, st = gp.solve([2.0])
    say("all fixed", precision, st)
    assert st["status"] == G.OK and st["iters"] == 1 and st["pcg_iters_total"] == 0
    np.testing.assert_array_equal(xg.cpu().numpy().astype(np.float64), m["rest_xyz"])
    ga, ast = gp.adjoint(np.ones((3, gp.n)))
    say("  adjoint", ast, ga.cpu().numpy())
    assert ast["status"] == G.OK and float(ga[0]) == 0.0


def test_mesh_without_chambers_solves_and_differentiates(G):
    m = voxel_box(2, 2, 1, h=1.0)
    m["fixed"][0] = 1
    gp = G.Problem(m["rest_xyz"], m["tets"], m["tet_mode"], m["tet_chamber"], m["fixed"], 0,
                   precision=8, self_collision=1, pcg_eta=1e-13, pcg_max=100)
    xg, st = gp.solve([])
    say("no chambers", st)
    assert st["status"] == G.OK
    np.testing.assert_allclose(xg.cpu().numpy(), m["rest_xyz"], atol=1e-12)
    ga, ast = gp.adjoint(np.ones((3, gp.n)))
    assert ast["status"] == G.OK and ga.numel() == 0


def test_fp32_adjoints_agree_in_both_cg_layouts(G, finger_oracle_150):
    """The adjoint kernels write the CG right-hand side in the layout of the
    grid they are given (three arrays of rows for the paired kernel, rows of
    three vectors otherwise). The same forward path (pcg_eta 1e-7, the contact
    rows of the oracle) differentiated on one block and on the default grid
    gives the same gradients to FP32 accuracy."""
    wl, prob, xo, orows = finger_oracle_150
    rng = np.random.default_rng(7)
    g = rng.standard_normal((3, prob.n))
    g[:, prob.fixed] = 0.0
    out = {}
    for blocks in (1, 0):
        gp = G.Problem.from_workload(wl, precision=4, pcg_eta=1e-7, pcg_max=3000, fixed_iters=150,
                                     pcg_blocks=blocks, adj_tol=1e-7, adj_aa_m=16)
        grid = gp.info["pcg_grid"]
        rows_per_block = ((gp.n + grid - 1) // grid + 63) // 64 * 64
        _, st = gp.solve(wl.alpha)
        np.testing.assert_array_equal(gp.contacts()["rows"], orows)
        ga, ast = gp.adjoint(g)
        gu, _, _, ust = gp.adjoint_unrolled(wl.alpha, 20, g)
        say("pcg_blocks", blocks, "grid", grid, "rows per block", rows_per_block, "adjoint", ast, "unrolled", ust)
        assert ast["status"] == G.OK
        out[blocks] = (ga.cpu().numpy().astype(np.float64), gu.cpu().numpy().astype(np.float64), rows_per_block)
    assert out[1][2] > 256 and out[0][2] <= 256  # unpaired, then paired
    for i, name in ((0, "implicit"), (1, "unrolled")):
        a, b = out[1][i], out[0][i]
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        say(name, "one block", a, "default grid", b, "rel", rel)
        assert rel < 1e-3
