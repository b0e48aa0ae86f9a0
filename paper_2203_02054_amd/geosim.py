"""Python binding of libgeosim (argument marshalling only).

Every step of the solve runs in the HIP library; PyTorch provides device
memory and the stream.  The binding fails loudly when the library is not
built or no GPU is present: there is no fallback path.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgeosim.so")

OK, NOT_CONVERGED = 0, 1
EINVAL, EDEGENERATE, EBREAKDOWN, ECAPACITY, ESTATE, EHIP = -1, -2, -3, -4, -5, -6
BODY, CH_ISO, CH_AX_X, CH_AX_Y, CH_AX_Z = 0, 1, 2, 3, 4
CONTACT_SELF, CONTACT_SPHERE, CONTACT_PLANE, CONTACT_MESH = 0, 1, 2, 3
AA_GUARD_NONE, AA_GUARD_RESIDUAL, AA_GUARD_ENERGY, AA_GUARD_SET = 0, 1, 2, 4


class GeosimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"geosim error {code}: {msg}")
        self.code = code


class MeshDesc(ctypes.Structure):
    _fields_ = [("n_verts", ctypes.c_int32), ("n_tets", ctypes.c_int32), ("n_chambers", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("rest_xyz", ctypes.c_void_p), ("tets", ctypes.c_void_p),
                ("tet_mode", ctypes.c_void_p), ("tet_chamber", ctypes.c_void_p), ("fixed", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("c1", ctypes.c_double), ("c2", ctypes.c_double), ("hyperelastic", ctypes.c_int32),
                ("kappa_col", ctypes.c_double), ("eps_rel", ctypes.c_double), ("ray_rel", ctypes.c_double),
                ("self_collision", ctypes.c_int32), ("obstacle_collision", ctypes.c_int32),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("fixed_iters", ctypes.c_int32),
                ("pcg_eta", ctypes.c_double), ("pcg_max", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("pcg_blocks", ctypes.c_int32), ("trace_len", ctypes.c_int32), ("adj_tol", ctypes.c_double),
                ("adj_max_iter", ctypes.c_int32), ("adj_aa_m", ctypes.c_int32), ("aa_m", ctypes.c_int32),
                ("aa_guard", ctypes.c_int32), ("aa_slack", ctypes.c_double), ("barrier_timeout_ms", ctypes.c_double),
                ("pcg_eta_min", ctypes.c_double), ("pcg_coarse", ctypes.c_int32), ("pcg_per_mesh", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("pcg_store", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("pcg_iters_total", ctypes.c_int32), ("n_contacts", ctypes.c_int32),
                ("ray_miss", ctypes.c_int32), ("residual", ctypes.c_double), ("energy", ctypes.c_double),
                ("aa_rejected", ctypes.c_int32), ("pad", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class Stage(ctypes.Structure):
    _fields_ = [("solve", Stats), ("status", ctypes.c_int32), ("n_flagged", ctypes.c_int32),
                ("alpha_top", ctypes.c_double)]

    def as_dict(self):
        return dict(solve=self.solve.as_dict(), status=self.status, n_flagged=self.n_flagged,
                    alpha_top=self.alpha_top)


class Info(ctypes.Structure):
    _fields_ = [("n_verts", ctypes.c_int32), ("n_tets", ctypes.c_int32), ("n_surface_faces", ctypes.c_int32),
                ("n_surface_verts", ctypes.c_int32), ("n_query_verts", ctypes.c_int32), ("nnz", ctypes.c_int32),
                ("n_slots", ctypes.c_int32), ("hash_buckets", ctypes.c_int32), ("h_ref", ctypes.c_double),
                ("eps_off", ctypes.c_double), ("ray_len", ctypes.c_double), ("bbox_diag", ctypes.c_double),
                ("cell_size", ctypes.c_double), ("ell_width", ctypes.c_int32), ("pcg_grid", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.c_void_p
_I = ctypes.c_int32
_PI = ctypes.POINTER(ctypes.c_int32)
_PD = ctypes.POINTER(ctypes.c_double)

# name -> (restype, argtypes); every entry point the header declares
SIGNATURES = {
    "gs_version": (_I, []),
    "gs_last_error": (ctypes.c_char_p, []),
    "gs_default_params": (None, [ctypes.POINTER(Params)]),
    "gs_create": (_I, [ctypes.POINTER(MeshDesc), ctypes.POINTER(Params), ctypes.POINTER(_P)]),
    "gs_set_obstacles": (_I, [_P, _I, _PD, _I, _PD]),
    "gs_set_mesh_obstacle": (_I, [_P, _I, _PD, _I, _PI]),
    "gs_info_get": (_I, [_P, ctypes.POINTER(Info)]),
    "gs_workspace_size": (_I, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "gs_bind": (_I, [_P, _P, ctypes.c_size_t, _P]),
    "gs_set_params": (_I, [_P, ctypes.POINTER(Params)]),
    "gs_solve": (_I, [_P, _P, _P, ctypes.POINTER(Stats)]),
    "gs_reset_contacts": (_I, [_P]),
    "gs_contacts": (_I, [_P, _I, _PI, _PI, _PI, _PD, _PD, _PI, _PI]),
    "gs_set_contacts": (_I, [_P, _I, _PI, _PI, _PI, _PD, _PD, _PI]),
    "gs_adjoint": (_I, [_P, _P, _P, _P, ctypes.POINTER(Stats)]),
    "gs_autotune": (_I, [_P, _P, _P, _I, _PI, _PD]),
    "gs_cg_plan": (_I, [_P, _I, _PI]),
    "gs_unrolled_scratch_size": (ctypes.c_size_t, [_P, _I]),
    "gs_adjoint_unrolled": (_I, [_P, _P, _P, _I, _P, _P, _P, _P, _P, ctypes.c_size_t, ctypes.POINTER(Stats)]),
    "gs_local_step_debug": (_I, [_P, _P, _P, _P]),
    "gs_tets": (_I, [_P, _PI]),
    "gs_faces": (_I, [_P, _PI]),
    "gs_collide_debug_scratch": (ctypes.c_size_t, [_I]),
    "gs_collide_debug": (_I, [_P, _P, _I, _P, ctypes.c_size_t, _PI, _PI, _PI, _PI, _PI, _PD, _PI]),
    "gs_collide_debug_static": (_I, [_P, _P, _I, _PI, _PI, _PI, _PI, _PI, _PD, _PI]),
    "gs_trace": (_I, [_P, _I, _PD, _PI]),
    "gs_tree_candidates_scratch": (ctypes.c_size_t, [_P, _I]),
    "gs_tree_candidates": (_I, [_P, _P, _I, _P, ctypes.c_size_t, _PI, _PI, _PD, _PD]),
    "gs_remesh_flags": (_I, [_P, _P, _P, ctypes.c_double, ctypes.c_double, _P, _PI]),
    "gs_solve_progressive": (_I, [_P, _P, _P, ctypes.c_double, ctypes.c_double, _I, _P, _I,
                                  ctypes.POINTER(Stage), _PI]),
    "gs_create_batch": (_I, [_I, ctypes.POINTER(MeshDesc), ctypes.POINTER(Params), ctypes.POINTER(_P)]),
    "gs_batch_layout": (_I, [_P, _I, _PI, _PI, _PI, _PI]),
    "gs_mesh_iters": (_I, [_P, _I, _PI]),
    "gs_profile": (_I, [_P, _I]),
    "gs_profile_read": (_I, [_P, _PD, ctypes.POINTER(ctypes.c_int64)]),
    "gs_kernel_name": (ctypes.c_char_p, [_I]),
    "gs_destroy": (None, [_P]),
}

N_KERNELS = 14

_lib = None

# Problems not yet closed.  They are closed at interpreter exit, before the
# HIP runtime tears itself down: a handle's destructor frees pinned host
# memory and events, which must not run after that teardown (nor from a
# finaliser during interpreter shutdown).
_live = weakref.WeakSet()


def _close_all():
    for p in list(_live):
        try:
            p.close()
        except Exception:
            pass


atexit.register(_close_all)


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2203_02054_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code, allow=(OK,)):
    if code in allow:
        return code
    raise GeosimError(code, lib().gs_last_error().decode())


def default_params(**kw) -> Params:
    p = Params()
    lib().gs_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, type(getattr(p, k))(v))
    return p


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("geosim needs a HIP GPU (torch.cuda.is_available() is False)")
    return torch


class Problem:
    """One tet mesh bound to a device workspace and a stream."""

    def __init__(self, rest_xyz, tets, tet_mode, tet_chamber, fixed, n_chambers, precision=4, params=None,
                 spheres=None, planes=None, device=None, stream=None, mesh_obstacle=None, **kw):
        self._setup([dict(rest_xyz=rest_xyz, tets=tets, tet_mode=tet_mode, tet_chamber=tet_chamber, fixed=fixed,
                          n_chambers=n_chambers)], precision, params, spheres, planes, device, stream, kw,
                    mesh_obstacle=mesh_obstacle)

    @classmethod
    def batch(cls, meshes, precision=4, params=None, spheres=None, planes=None, device=None, stream=None,
              mesh_obstacle=None, **kw):
        """Several meshes solved together (dicts with the Problem arguments, or
        workloads); arrays are concatenated in mesh order."""
        self = cls.__new__(cls)
        ms = []
        for m in meshes:
            if not isinstance(m, dict):
                m = dict(rest_xyz=m.rest_xyz, tets=m.tets, tet_mode=m.tet_mode, tet_chamber=m.tet_chamber,
                         fixed=m.fixed, n_chambers=m.n_chambers)
            ms.append(m)
        self._setup(ms, precision, params, spheres, planes, device, stream, kw, batch=True,
                    mesh_obstacle=mesh_obstacle)
        return self

    def _setup(self, meshes, precision, params, spheres, planes, device, stream, kw, batch=False,
               mesh_obstacle=None):
        torch = _torch()
        self.torch = torch
        self.device = torch.device(device or "cuda")
        self.dtype = torch.float32 if precision == 4 else torch.float64
        self.np_dtype = np.float32 if precision == 4 else np.float64
        self._keep = []
        descs = (MeshDesc * len(meshes))()
        for i, m in enumerate(meshes):
            X = np.ascontiguousarray(m["rest_xyz"], dtype=np.float64)
            T = np.ascontiguousarray(m["tets"], dtype=np.int32)
            md = np.ascontiguousarray(m["tet_mode"], dtype=np.uint8)
            ch = np.ascontiguousarray(m["tet_chamber"], dtype=np.int16)
            fx = np.ascontiguousarray(m["fixed"], dtype=np.uint8)
            self._keep += [X, T, md, ch, fx]
            descs[i] = MeshDesc(X.shape[1], T.shape[1], int(m["n_chambers"]), int(precision), X.ctypes.data,
                                T.ctypes.data, md.ctypes.data, ch.ctypes.data, fx.ctypes.data)
        self._X = np.concatenate([np.asarray(m["rest_xyz"], dtype=np.float64) for m in meshes], axis=1)
        self.n = self._X.shape[1]
        self.T = sum(int(np.asarray(m["tets"]).shape[1]) for m in meshes)
        self.n_chambers = sum(int(m["n_chambers"]) for m in meshes)
        self.n_mesh = len(meshes)
        self.params = params if params is not None else default_params(**kw)
        h = _P()
        if batch:
            _check(lib().gs_create_batch(len(meshes), descs, ctypes.byref(self.params), ctypes.byref(h)))
        else:
            _check(lib().gs_create(ctypes.byref(descs[0]), ctypes.byref(self.params), ctypes.byref(h)))
        self._h = h
        self.state_id = 0   # bumped by every call that replaces the solved state
        _live.add(self)
        sph = np.ascontiguousarray(np.zeros((0, 4)) if spheres is None else spheres, dtype=np.float64).reshape(-1, 4)
        pln = np.ascontiguousarray(np.zeros((0, 6)) if planes is None else planes, dtype=np.float64).reshape(-1, 6)
        if sph.shape[0] or pln.shape[0]:
            _check(lib().gs_set_obstacles(h, sph.shape[0], _ptr(sph, ctypes.c_double), pln.shape[0],
                                          _ptr(pln, ctypes.c_double)))
        if mesh_obstacle is not None:
            mv = np.ascontiguousarray(mesh_obstacle[0], dtype=np.float64)
            mt = np.ascontiguousarray(np.asarray(mesh_obstacle[1]).T, dtype=np.int32)   # [3][k]
            _check(lib().gs_set_mesh_obstacle(h, mv.shape[1], _ptr(mv, ctypes.c_double), mt.shape[1],
                                              _ptr(mt, ctypes.c_int32)))
        nb = ctypes.c_size_t()
        _check(lib().gs_workspace_size(h, ctypes.byref(nb)))
        self.ws_bytes = nb.value
        self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(lib().gs_bind(h, self._ws_ptr, self.ws_bytes, self.stream.cuda_stream))
        inf = Info()
        _check(lib().gs_info_get(h, ctypes.byref(inf)))
        self.info = inf.as_dict()

    def layout(self):
        """Per-mesh offsets: dict of vert/tet/chamber offset arrays [n_mesh + 1]."""
        cap = self.n_mesh + 1
        v, t, c = (np.zeros(cap, np.int32) for _ in range(3))
        nm = ctypes.c_int32()
        _check(lib().gs_batch_layout(self._h, cap, _ptr(v, ctypes.c_int32), _ptr(t, ctypes.c_int32),
                                     _ptr(c, ctypes.c_int32), ctypes.byref(nm)))
        return dict(vert=v, tet=t, chamber=c)

    def cg_plan(self):
        """Workgroups of the per-mesh CG for each mesh (all 1 without it)."""
        k = np.zeros(self.n_mesh, np.int32)
        _check(lib().gs_cg_plan(self._h, self.n_mesh, _ptr(k, ctypes.c_int32)))
        return k

    def mesh_iters(self):
        it = np.zeros(self.n_mesh, np.int32)
        _check(lib().gs_mesh_iters(self._h, self.n_mesh, _ptr(it, ctypes.c_int32)))
        return it

    @classmethod
    def from_workload(cls, wl, precision=None, **kw):
        for k, v in getattr(wl, "solver", {}).items():
            kw.setdefault(k, v)
        kw.setdefault("c1", wl.material[0])
        kw.setdefault("c2", wl.material[1])
        kw.setdefault("self_collision", int(wl.self_collision))
        kw.setdefault("obstacle_collision", int(wl.obstacle_collision))
        kw.setdefault("fixed_iters", wl.fixed_iters)
        return cls(wl.rest_xyz, wl.tets, wl.tet_mode, wl.tet_chamber, wl.fixed, wl.n_chambers,
                   precision=precision or wl.precision, spheres=wl.spheres, planes=wl.planes,
                   mesh_obstacle=getattr(wl, "mesh_obstacle", None), **kw)

    # -- helpers -----------------------------------------------------------
    def tensor(self, a):
        t = self.torch.as_tensor(np.asarray(a), dtype=self.dtype)
        return t.to(self.device).contiguous()

    def _dev(self, t, shape):
        if not (t.is_cuda and t.dtype == self.dtype and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
            raise ValueError(f"expected a contiguous {self.dtype} device tensor of shape {shape}")
        return t.data_ptr()

    def close(self):
        """Release the library handle (idempotent).  The workspace tensor is
        released with the object."""
        if getattr(self, "_h", None):
            lib().gs_destroy(self._h)
            self._h = None
        _live.discard(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the atexit hook has closed every live handle;
        # a finaliser that still runs then must not call into the runtime (the
        # check is bound at definition: module globals may be gone by then)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    # -- entry points --------------------------------------------------------
    def set_params(self, **kw):
        for k, v in kw.items():
            if not hasattr(self.params, k):
                raise TypeError(f"unknown parameter {k}")
            setattr(self.params, k, type(getattr(self.params, k))(v))
        _check(lib().gs_set_params(self._h, ctypes.byref(self.params)))
        inf = Info()
        _check(lib().gs_info_get(self._h, ctypes.byref(inf)))
        self.info = inf.as_dict()

    def solve(self, alpha, x=None, allow_not_converged=True):
        """Solve from x (default: rest positions) with the stored contact set.
        Returns (x [3,n] device tensor, stats dict with 'status')."""
        a = alpha if self.torch.is_tensor(alpha) else self.tensor(np.asarray(alpha, dtype=np.float64).reshape(-1))
        if x is None:
            x = self.tensor(self._X)
        st = Stats()
        allow = (OK, NOT_CONVERGED) if allow_not_converged else (OK,)
        self.state_id += 1
        code = lib().gs_solve(self._h, self._dev(a, (self.n_chambers,)) if self.n_chambers else None,
                              self._dev(x, (3, self.n)), ctypes.byref(st))
        _check(code, allow)
        d = st.as_dict()
        d["status"] = code
        return x, d

    def adjoint_unrolled(self, alpha, K, dLdx, x0=None):
        """Unrolled gradient of L(x_K) over K iterations from x0 (default: rest)
        with the stored contact set as the previous one.  Returns
        (dL/dalpha, dL/dx0, x_K, stats dict) as device tensors."""
        a = alpha if self.torch.is_tensor(alpha) else self.tensor(np.asarray(alpha, dtype=np.float64).reshape(-1))
        if x0 is None:
            x0 = self.tensor(self._X)
        g = dLdx if self.torch.is_tensor(dLdx) else self.tensor(np.asarray(dLdx, dtype=np.float64))
        nb = int(lib().gs_unrolled_scratch_size(self._h, int(K)))
        scratch = self.torch.empty(nb + 256, dtype=self.torch.uint8, device=self.device)
        sp = (scratch.data_ptr() + 255) & ~255
        ga = self.torch.zeros(max(self.n_chambers, 1), dtype=self.dtype, device=self.device)[:self.n_chambers]
        gx0 = self.torch.empty((3, self.n), dtype=self.dtype, device=self.device)
        xK = self.torch.empty((3, self.n), dtype=self.dtype, device=self.device)
        st = Stats()
        self.state_id += 1
        _check(lib().gs_adjoint_unrolled(self._h, self._dev(a, (self.n_chambers,)) if self.n_chambers else None,
                                         self._dev(x0, (3, self.n)), int(K), self._dev(g, (3, self.n)),
                                         ga.data_ptr() if self.n_chambers else None, gx0.data_ptr(),
                                         xK.data_ptr(), sp, nb, ctypes.byref(st)))
        return ga, gx0, xK, st.as_dict()

    def autotune(self, alpha, x=None, iters=20):
        """Pick the CG grid by timing `iters` fixed iterations per candidate from
        x (default: rest positions); returns (grid, ms per outer iteration)."""
        a = alpha if self.torch.is_tensor(alpha) else self.tensor(np.asarray(alpha, dtype=np.float64).reshape(-1))
        if x is None:
            x = self.tensor(self._X)
        g = ctypes.c_int32()
        ms = ctypes.c_double()
        self.state_id += 1
        _check(lib().gs_autotune(self._h, self._dev(a, (self.n_chambers,)) if self.n_chambers else None,
                                 self._dev(x, (3, self.n)), int(iters), ctypes.byref(g), ctypes.byref(ms)))
        self.params.pcg_blocks = g.value
        inf = Info()
        _check(lib().gs_info_get(self._h, ctypes.byref(inf)))
        self.info = inf.as_dict()
        return g.value, ms.value

    def trace(self):
        """Per-iteration rows (r_k, E_k, springs, changed, CG its, ray misses) of the last solve."""
        cap = max(self.params.trace_len, 1)
        out = np.zeros((cap, 6))
        cnt = ctypes.c_int32()
        _check(lib().gs_trace(self._h, cap, _ptr(out, ctypes.c_double), ctypes.byref(cnt)))
        return out[:cnt.value]

    def profile(self, enable=True):
        _check(lib().gs_profile(self._h, int(enable)))

    def profile_read(self):
        """{kernel name: (total ms, launches)} since profiling was enabled."""
        ms = np.zeros(N_KERNELS)
        cnt = np.zeros(N_KERNELS, np.int64)
        _check(lib().gs_profile_read(self._h, _ptr(ms, ctypes.c_double), _ptr(cnt, ctypes.c_int64)))
        return {lib().gs_kernel_name(k).decode(): (float(ms[k]), int(cnt[k])) for k in range(N_KERNELS)}

    def reset_contacts(self):
        self.state_id += 1
        _check(lib().gs_reset_contacts(self._h))

    def contacts(self):
        m = self.info["n_query_verts"] * self.info["n_slots"]
        cap = max(m, 1)
        v, t, p, fr = (np.zeros(cap, np.int32) for _ in range(4))
        tg, nr = np.zeros((cap, 3)), np.zeros((cap, 3))
        cnt = ctypes.c_int32()
        _check(lib().gs_contacts(self._h, cap, _ptr(v, ctypes.c_int32), _ptr(t, ctypes.c_int32),
                                 _ptr(p, ctypes.c_int32), _ptr(tg, ctypes.c_double), _ptr(nr, ctypes.c_double),
                                 _ptr(fr, ctypes.c_int32), ctypes.byref(cnt)))
        k = cnt.value
        return dict(rows=np.stack([v[:k], t[:k], p[:k]], axis=1), target=tg[:k], normal=nr[:k],
                    fresh=fr[:k].astype(bool))

    def set_contacts(self, rows, target, normal, fresh=None):
        rows = np.ascontiguousarray(rows, dtype=np.int32).reshape(-1, 3)
        v, t, p = (np.ascontiguousarray(rows[:, i]) for i in range(3))
        tg = np.ascontiguousarray(target, dtype=np.float64).reshape(-1, 3)
        nr = np.ascontiguousarray(normal, dtype=np.float64).reshape(-1, 3)
        fr = None if fresh is None else np.ascontiguousarray(fresh, dtype=np.int32).reshape(-1)
        self.state_id += 1
        _check(lib().gs_set_contacts(self._h, rows.shape[0], _ptr(v, ctypes.c_int32), _ptr(t, ctypes.c_int32),
                                     _ptr(p, ctypes.c_int32), _ptr(tg, ctypes.c_double), _ptr(nr, ctypes.c_double),
                                     None if fr is None else _ptr(fr, ctypes.c_int32)))

    def adjoint(self, dLdx, want_mu=False, allow_not_converged=True):
        """Implicit adjoint of the last solve for dL/dx [3, n] (device tensor or
        array): returns (dL/dalpha [n_chambers] device tensor, stats dict[, mu])."""
        g = dLdx if self.torch.is_tensor(dLdx) else self.tensor(np.asarray(dLdx, dtype=np.float64))
        out = self.torch.zeros(max(self.n_chambers, 1), dtype=self.dtype, device=self.device)[:self.n_chambers]
        mu = self.torch.empty((3, self.n), dtype=self.dtype, device=self.device) if want_mu else None
        st = Stats()
        code = lib().gs_adjoint(self._h, self._dev(g, (3, self.n)), out.data_ptr() if self.n_chambers else None,
                                mu.data_ptr() if want_mu else None, ctypes.byref(st))
        _check(code, (OK, NOT_CONVERGED) if allow_not_converged else (OK,))
        d = st.as_dict()
        d["status"] = code
        return (out, d, mu) if want_mu else (out, d)

    def local_step(self, x, alpha):
        """Centred target shapes [3, 4, T] at positions x."""
        a = alpha if self.torch.is_tensor(alpha) else self.tensor(np.asarray(alpha, dtype=np.float64).reshape(-1))
        out = self.torch.empty((3, 4, self.T), dtype=self.dtype, device=self.device)
        _check(lib().gs_local_step_debug(self._h, self._dev(x, (3, self.n)),
                                         self._dev(a, (self.n_chambers,)) if self.n_chambers else None,
                                         out.data_ptr()))
        self.stream.synchronize()
        return out

    def oriented_tets(self):
        t = np.zeros((4, self.T), np.int32)
        _check(lib().gs_tets(self._h, _ptr(t, ctypes.c_int32)))
        return t

    def faces(self):
        f = np.zeros((3, self.info["n_surface_faces"]), np.int32)
        _check(lib().gs_faces(self._h, _ptr(f, ctypes.c_int32)))
        return f

    def remesh_flags(self, x, x_ref=None, alpha_max=4.0, d_max=4.0):
        """Remesh checks of the chamber elements at x against x_ref (default:
        the rest shape).  Returns (flags uint8 device tensor [T] in the order
        of oriented_tets, number flagged)."""
        flags = self.torch.empty(self.T, dtype=self.torch.uint8, device=self.device)
        nf = ctypes.c_int32()
        _check(lib().gs_remesh_flags(self._h, self._dev(x, (3, self.n)),
                                     None if x_ref is None else self._dev(x_ref, (3, self.n)),
                                     float(alpha_max), float(d_max), flags.data_ptr(), ctypes.byref(nf)))
        return flags, nf.value

    def solve_progressive(self, alpha, x=None, alpha_max=4.0, d_max=4.0, stop_on_flag=True, cap=64):
        """Progressive actuation: stages alpha_k = min(alpha, (k+1) alpha_max),
        each a solve warm-started from the last, then the remesh checks.
        Returns (x, flags uint8 [T], list of stage dicts, status)."""
        a = alpha if self.torch.is_tensor(alpha) else self.tensor(np.asarray(alpha, dtype=np.float64).reshape(-1))
        if x is None:
            x = self.tensor(self._X)
        flags = self.torch.empty(self.T, dtype=self.torch.uint8, device=self.device)
        stages = (Stage * cap)()
        ns = ctypes.c_int32()
        self.state_id += 1
        code = lib().gs_solve_progressive(self._h, self._dev(a, (self.n_chambers,)) if self.n_chambers else None,
                                          self._dev(x, (3, self.n)), float(alpha_max), float(d_max),
                                          int(bool(stop_on_flag)), flags.data_ptr(), cap, stages, ctypes.byref(ns))
        _check(code, (OK, NOT_CONVERGED))
        return x, flags, [stages[i].as_dict() for i in range(ns.value)], code

    def tree_candidates(self, x, cap=None):
        """C_tet at x from the refit-only tet tree: (pairs [k, 2] sorted by
        (v, e), refit ms, query ms)."""
        cap = int(cap or max(4 * self.info["n_query_verts"] * 8, 1024))
        nb = int(lib().gs_tree_candidates_scratch(self._h, cap))
        scratch = self.torch.empty(nb + 256, dtype=self.torch.uint8, device=self.device)
        sp = (scratch.data_ptr() + 255) & ~255
        out = np.zeros((2, cap), np.int32)
        cnt = ctypes.c_int32()
        t1, t2 = ctypes.c_double(), ctypes.c_double()
        code = lib().gs_tree_candidates(self._h, self._dev(x, (3, self.n)), cap, sp, nb, _ptr(out, ctypes.c_int32),
                                        ctypes.byref(cnt), ctypes.byref(t1), ctypes.byref(t2))
        if code == ECAPACITY:
            return self.tree_candidates(x, cap=2 * max(cap, cnt.value))
        _check(code)
        return out[:, :cnt.value].T.copy(), t1.value, t2.value

    def collide(self, x, cap=None):
        """One collision check at x with the stored set as the previous one."""
        cap = int(cap or max(4 * self.info["n_query_verts"] * 8, 1024))
        nbytes = lib().gs_collide_debug_scratch(cap)
        scratch = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device)
        ct, tr, co = np.zeros((2, cap), np.int32), np.zeros((2, cap), np.int32), np.zeros((3, cap), np.int32)
        tg = np.zeros((3, cap))
        nct, ntr, nco = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        code = lib().gs_collide_debug(self._h, self._dev(x, (3, self.n)), cap, scratch.data_ptr(), nbytes,
                                      _ptr(ct, ctypes.c_int32), ctypes.byref(nct), _ptr(tr, ctypes.c_int32),
                                      ctypes.byref(ntr), _ptr(co, ctypes.c_int32), _ptr(tg, ctypes.c_double),
                                      ctypes.byref(nco))
        if code == ECAPACITY:
            return self.collide(x, cap=2 * max(cap, nct.value, ntr.value, nco.value))
        _check(code)
        a, b, k = nct.value, ntr.value, nco.value
        return dict(cand_tet=ct[:, :a].T.copy(), cand_tri=tr[:, :b].T.copy(), contacts=co[:, :k].T.copy(),
                    target=tg[:, :k].T.copy())


STATIC_CAND_CAP = 131072


def _collide_static(self, x, cap=None):
    """gs_collide_debug_static: one collision check at x staged in the
    library's static device array (no allocation); cap <= STATIC_CAND_CAP."""
    cap = int(cap if cap is not None else STATIC_CAND_CAP)
    ct, tr, co = np.zeros((2, cap), np.int32), np.zeros((2, cap), np.int32), np.zeros((3, cap), np.int32)
    tg = np.zeros((3, cap))
    nct, ntr, nco = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().gs_collide_debug_static(self._h, self._dev(x, (3, self.n)), cap, _ptr(ct, ctypes.c_int32),
                                         ctypes.byref(nct), _ptr(tr, ctypes.c_int32), ctypes.byref(ntr),
                                         _ptr(co, ctypes.c_int32), _ptr(tg, ctypes.c_double), ctypes.byref(nco)))
    a, b, k = nct.value, ntr.value, nco.value
    return dict(cand_tet=ct[:, :a].T.copy(), cand_tri=tr[:, :b].T.copy(), contacts=co[:, :k].T.copy(),
                target=tg[:, :k].T.copy())


Problem.collide_static = _collide_static


class _SolveFn:
    """Holder for the autograd function (built lazily so importing this module
    does not import torch)."""
    fn = None


def solve_fn():
    """torch.autograd.Function: x = SolveFn.apply(alpha, problem, x0).

    Forward runs gs_solve from x0 (rest positions when None) with the stored
    contact set and raises unless it converged (the implicit gradient is
    defined only at a fixed point); backward runs gs_adjoint on the incoming
    dL/dx and returns dL/dalpha (implicit gradient at the solve's fixed point
    with its contact set held fixed).  The gradient is taken of the state the
    problem holds, so backward raises if anything replaced that state since
    this forward (another solve, an autotune, an unrolled adjoint, contacts
    set or reset); it warns if the adjoint iteration hit its cap."""
    if _SolveFn.fn is None:
        import warnings

        import torch

        class SolveFn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, alpha, problem, x0=None):
                x = problem.tensor(problem._X) if x0 is None else x0.detach().clone().contiguous()
                problem.solve(alpha.detach().contiguous(), x, allow_not_converged=False)
                ctx.problem = problem
                ctx.state_id = problem.state_id
                return x

            @staticmethod
            def backward(ctx, gx):
                if ctx.problem.state_id != ctx.state_id:
                    raise RuntimeError("the problem was solved again (or its state replaced) after this "
                                       "forward: its adjoint would differentiate another state")
                ga, st = ctx.problem.adjoint(gx.detach().to(ctx.problem.dtype).contiguous())
                if st["status"] != OK:
                    warnings.warn(f"adjoint iteration did not converge (residual {st['residual']:.3e})")
                return ga, None, None

        _SolveFn.fn = SolveFn
    return _SolveFn.fn
