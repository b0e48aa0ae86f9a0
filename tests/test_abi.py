"""The C ABI without a GPU: exported symbols, host-side validation and the
once-per-mesh set-up (orientation, boundary faces, query vertices, sizes),
checked against the oracle's set-up."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2203_02054_amd import geosim as G
from paper_2203_02054_amd import meshgen as mg
import oracle
from tests.meshes import voxel_box

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "geosim.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported_and_bound():
    L = G.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert sorted(G.SIGNATURES) == names
    assert L.gs_version() == 211


def _desc(m, precision=4):
    keep = dict(X=np.ascontiguousarray(m["rest_xyz"], np.float64), T=np.ascontiguousarray(m["tets"], np.int32),
                M=np.ascontiguousarray(m["tet_mode"], np.uint8), C=np.ascontiguousarray(m["tet_chamber"], np.int16),
                F=np.ascontiguousarray(m["fixed"], np.uint8))
    d = G.MeshDesc(keep["X"].shape[1], keep["T"].shape[1], int(m.get("n_chambers", 1)), precision,
                   keep["X"].ctypes.data, keep["T"].ctypes.data, keep["M"].ctypes.data, keep["C"].ctypes.data,
                   keep["F"].ctypes.data)
    return d, keep


def _create(m, **kw):
    d, keep = _desc(m)
    p = G.default_params(**kw)
    h = ctypes.c_void_p()
    code = G.lib().gs_create(ctypes.byref(d), ctypes.byref(p), ctypes.byref(h))
    return code, h, keep


def test_create_rejects_bad_input():
    m = voxel_box(2, 1, 1)
    bad = dict(m, tets=m["tets"].copy())
    bad["tets"][0, 0] = 10_000
    assert _create(bad)[0] == G.EINVAL
    nan = dict(m, rest_xyz=m["rest_xyz"].copy())
    nan["rest_xyz"][1, 3] = np.nan
    assert _create(nan)[0] == G.EINVAL
    flat = dict(m, rest_xyz=m["rest_xyz"].copy())
    flat["rest_xyz"][2] = 0.0                      # every tet flat
    assert _create(flat)[0] == G.EDEGENERATE
    ch = dict(m, tet_mode=np.full(m["tets"].shape[1], G.CH_ISO, np.uint8))   # chamber id -1
    assert _create(ch)[0] == G.EINVAL
    assert _create(m, pcg_eta=0.0)[0] == G.EINVAL
    assert _create(m, c1=-1.0)[0] == G.EINVAL
    code, h, _ = _create(m)
    assert code == G.OK
    st = G.Stats()
    assert G.lib().gs_solve(h, None, None, ctypes.byref(st)) == G.ESTATE       # not bound
    sph = np.array([0.0, 0.0, 0.0, -1.0])
    assert G.lib().gs_set_obstacles(h, 1, sph.ctypes.data_as(G._PD), 0, None) == G.EINVAL
    pl = np.array([0.0, 0.0, 0.0, 0.0, 0.0, 0.0])
    assert G.lib().gs_set_obstacles(h, 0, None, 1, pl.ctypes.data_as(G._PD)) == G.EINVAL
    assert "normal" in G.lib().gs_last_error().decode()
    G.lib().gs_destroy(h)


@pytest.mark.parametrize("name", ["block", "finger_small"])
def test_host_setup_matches_oracle(name):
    wl = mg.make("block") if name == "block" else mg.finger(4.0, 3, 2.0)
    prob = oracle.Problem.from_workload(wl)
    m = dict(rest_xyz=wl.rest_xyz, tets=wl.tets, tet_mode=wl.tet_mode, tet_chamber=wl.tet_chamber,
             fixed=wl.fixed, n_chambers=wl.n_chambers)
    code, h, keep = _create(m)
    assert code == G.OK
    info = G.Info()
    G.lib().gs_info_get(h, ctypes.byref(info))
    assert info.n_tets == prob.T and info.n_verts == prob.n
    assert info.n_surface_faces == prob.faces.shape[0]
    assert info.n_surface_verts == prob.surf_verts.size
    assert info.n_query_verts == prob.query_verts.size
    assert info.h_ref == pytest.approx(prob.h_ref, rel=1e-12)
    assert info.bbox_diag == pytest.approx(prob.diag, rel=1e-12)
    assert info.eps_off == pytest.approx(prob.eps_off, rel=1e-12)
    # Dirichlet-reduced CSR: free-free entries of A_el plus one diagonal per fixed row
    F = prob.free
    red = prob.A_el[F][:, F]
    assert info.nnz == red.nnz + int(prob.fixed.sum())
    t = np.zeros((4, prob.T), np.int32)
    G.lib().gs_tets(h, t.ctypes.data_as(G._PI))
    np.testing.assert_array_equal(t, prob.tets)
    f = np.zeros((3, info.n_surface_faces), np.int32)
    G.lib().gs_faces(h, f.ctypes.data_as(G._PI))
    np.testing.assert_array_equal(f.T, prob.faces)
    nb = ctypes.c_size_t()
    G.lib().gs_workspace_size(h, ctypes.byref(nb))
    assert nb.value > 0
    G.lib().gs_destroy(h)


def test_batch_setup_concatenates_meshes():
    """A batch is the meshes concatenated: its sizes are the sums of the single-mesh
    set-ups and each mesh's oriented tets and faces are offset copies."""
    wls = [mg.finger(4.0, 3, 2.0), mg.make("block"), mg.finger(4.0, 4, 1.5)]
    probs = [oracle.Problem.from_workload(w) for w in wls]
    keep = []
    descs = (G.MeshDesc * len(wls))()
    for i, w in enumerate(wls):
        d, k = _desc(dict(rest_xyz=w.rest_xyz, tets=w.tets, tet_mode=w.tet_mode, tet_chamber=w.tet_chamber,
                          fixed=w.fixed, n_chambers=w.n_chambers))
        keep.append(k)
        descs[i] = d
    p = G.default_params()
    h = ctypes.c_void_p()
    assert G.lib().gs_create_batch(len(wls), descs, ctypes.byref(p), ctypes.byref(h)) == G.OK
    info = G.Info()
    G.lib().gs_info_get(h, ctypes.byref(info))
    assert info.n_tets == sum(q.T for q in probs)
    assert info.n_verts == sum(q.n for q in probs)
    assert info.n_surface_faces == sum(q.faces.shape[0] for q in probs)
    assert info.n_query_verts == sum(q.query_verts.size for q in probs)
    vo = np.zeros(4, np.int32)
    to = np.zeros(4, np.int32)
    co = np.zeros(4, np.int32)
    nm = ctypes.c_int32()
    assert G.lib().gs_batch_layout(h, 4, vo.ctypes.data_as(G._PI), to.ctypes.data_as(G._PI),
                                   co.ctypes.data_as(G._PI), ctypes.byref(nm)) == G.OK
    assert nm.value == 3
    np.testing.assert_array_equal(np.diff(vo), [q.n for q in probs])
    np.testing.assert_array_equal(np.diff(co), [w.n_chambers for w in wls])
    t = np.zeros((4, info.n_tets), np.int32)
    G.lib().gs_tets(h, t.ctypes.data_as(G._PI))
    f = np.zeros((3, info.n_surface_faces), np.int32)
    G.lib().gs_faces(h, f.ctypes.data_as(G._PI))
    fo = 0
    for m, q in enumerate(probs):
        np.testing.assert_array_equal(t[:, to[m]:to[m + 1]], q.tets + vo[m])
        nf = q.faces.shape[0]
        np.testing.assert_array_equal(f[:, fo:fo + nf].T, q.faces + vo[m])
        fo += nf
    G.lib().gs_destroy(h)


def test_acceleration_and_barrier_parameters_are_validated():
    m = voxel_box(2, 1, 1)
    for kw in (dict(aa_m=-1), dict(aa_m=17), dict(aa_guard=3), dict(aa_guard=8), dict(aa_slack=-0.1),
               dict(aa_slack=float("nan")), dict(barrier_timeout_ms=-1.0)):
        assert _create(m, **kw)[0] == G.EINVAL, kw
    code, h, _ = _create(m, aa_m=16, aa_guard=G.AA_GUARD_ENERGY, aa_slack=0.0, barrier_timeout_ms=0.0)
    assert code == G.OK
    G.lib().gs_destroy(h)
    p = G.default_params()
    assert (p.aa_m, p.aa_guard, p.aa_slack, p.barrier_timeout_ms) == (
        8, G.AA_GUARD_RESIDUAL | G.AA_GUARD_SET, 0.5, 2000.0)


def test_energy_guard_is_refused_for_a_batch():
    m = voxel_box(2, 1, 1)
    d0, k0 = _desc(m)
    d1, k1 = _desc(m)
    descs = (G.MeshDesc * 2)(d0, d1)
    h = ctypes.c_void_p()
    p = G.default_params(aa_guard=G.AA_GUARD_ENERGY)
    assert G.lib().gs_create_batch(2, descs, ctypes.byref(p), ctypes.byref(h)) == G.EINVAL
    p = G.default_params(aa_guard=G.AA_GUARD_ENERGY, aa_m=0)
    assert G.lib().gs_create_batch(2, descs, ctypes.byref(p), ctypes.byref(h)) == G.OK
    G.lib().gs_destroy(h)


def test_remesh_and_progressive_entry_points_validate_on_the_host():
    L = G.lib()
    st = (G.Stage * 4)()
    n = ctypes.c_int32()
    assert L.gs_remesh_flags(None, None, None, 4.0, 4.0, None, None) == G.EINVAL
    assert L.gs_solve_progressive(None, None, None, 4.0, 4.0, 1, None, 4, st, ctypes.byref(n)) == G.EINVAL
    code, h, keep = _create(voxel_box(2, 1, 1))
    assert code == G.OK
    try:
        # not bound to a device: refused before any device work
        assert L.gs_remesh_flags(h, None, None, 4.0, 4.0, None, None) == G.ESTATE
        assert L.gs_solve_progressive(h, None, None, 4.0, 4.0, 1, None, 4, st, ctypes.byref(n)) == G.ESTATE
    finally:
        L.gs_destroy(h)
    assert ctypes.sizeof(G.Stage) == ctypes.sizeof(G.Stats) + 16


def test_per_mesh_cg_parameter_and_plan_validate_on_the_host():
    m = voxel_box(2, 1, 1)
    for v in (-1, 3):
        assert _create(m, pcg_per_mesh=v)[0] == G.EINVAL, v
    code, h, _ = _create(m, pcg_per_mesh=2)
    assert code == G.OK
    G.lib().gs_destroy(h)
    assert G.default_params().pcg_per_mesh == 0
    L = G.lib()
    k = (ctypes.c_int32 * 1)()
    assert L.gs_cg_plan(None, 1, k) == G.EINVAL
    code, h, keep = _create(m, pcg_per_mesh=1)
    assert code == G.OK
    try:
        assert L.gs_cg_plan(h, 1, None) == G.EINVAL
        assert L.gs_cg_plan(h, 1, k) == G.ESTATE  # not bound to a device
    finally:
        L.gs_destroy(h)


def test_graph_and_store_parameters_are_validated():
    m = voxel_box(2, 1, 1)
    for kw in (dict(graph=-1), dict(graph=2), dict(pcg_store=-1), dict(pcg_store=3)):
        assert _create(m, **kw)[0] == G.EINVAL, kw
    p = G.default_params()
    assert (p.graph, p.pcg_store) == (0, 0)
