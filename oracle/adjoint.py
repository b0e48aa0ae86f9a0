"""Oracle gradients with respect to the chamber volume ratios: implicit
(at the local/global fixed point) and unrolled (through K iterations).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper has no gradient; this is the differentiable reading of its method.
At a fixed point x of the local/global iteration (Section III-B) with the
active contact set A held fixed, the free coordinates satisfy

    M_FF x_F = b_F(x, alpha) - M_FC x_C,

with M = A_el + diag(springs) and b the right-hand side of the global step:
the element targets of Section III-A (chamber rule, Eq. 6 blend, Eq. 7
volume scaling) and the spring targets of Section II-C, all functions of the
current positions.  Differentiating,

    (M_FF - db_F/dx_F) dx_F = (db_F/dalpha) dalpha,

so a loss L(x) with g = dL/dx has

    dL/dalpha = (db_F/dalpha)^T mu,    (M_FF - db_F/dx_F)^T mu = g_F.

Spring targets as functions of x (the collision response, Eq. 5 and Eq. 8):
  * a self contact given a new target at this iteration (the vertex
    penetrates and its ray hits face f): c = x_v + (t + eps) d with
    d = -n_v / |n_v| (n_v the sum of the cross products of the vertex's
    boundary faces) and t the Moller-Trumbore distance to f; it depends on
    x_v, on the vertices of v's boundary faces and on those of f;
  * a self contact kept from the previous iteration: its stored target, a
    constant;
  * sphere (c0, r): c = c0 + (r + eps) (x_v - c0) / |x_v - c0|;
  * plane (p, n): c = x_v - (n.(x_v - p) - eps) n.

The Kabsch rotation R of M = D Q^T is differentiated as a polar factor: with
S = R^T M symmetric, dR = R [w]x where (tr(S) I - S) w = vee(R^T dM - dM^T R)
(vee of a skew matrix Y is (Y32, Y13, Y21)).

Everything here is FP64.  The linear system for mu is solved by GMRES
preconditioned with the sparse factorisation of M_FF (library routines as
steps), to a residual of 1e-13 relative to g.  ``frozen_solve`` finds the
fixed point of the same frozen-set map (Anderson acceleration, Walker & Ni
2011, which leaves the fixed point unchanged) for finite-difference checks.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla
import torch

from .collision import Contacts, _incidence
from .local import kabsch, targets_torch, tensors
from .solver import system


class _PolarRotation(torch.autograd.Function):
    """Kabsch rotation with the polar-factor derivative (batched 3x3)."""

    @staticmethod
    def forward(ctx, M):
        with torch.no_grad():
            R = kabsch(M)
        ctx.save_for_backward(M, R)
        return R

    @staticmethod
    def backward(ctx, gR):
        M, R = ctx.saved_tensors
        S = R.transpose(-1, -2) @ M
        S = 0.5 * (S + S.transpose(-1, -2))
        tr = S.diagonal(dim1=-2, dim2=-1).sum(-1)
        K = tr[..., None, None] * torch.eye(3, dtype=M.dtype) - S
        A = R.transpose(-1, -2) @ gR
        a = torch.stack([A[..., 2, 1] - A[..., 1, 2], A[..., 0, 2] - A[..., 2, 0],
                         A[..., 1, 0] - A[..., 0, 1]], dim=-1)
        z = torch.linalg.solve(K, a[..., None])[..., 0]
        return R @ skew(z)


def skew(z: torch.Tensor) -> torch.Tensor:
    """[z]x such that [z]x y = z x y."""
    o = torch.zeros_like(z[..., 0])
    return torch.stack([torch.stack([o, -z[..., 2], z[..., 1]], -1),
                        torch.stack([z[..., 2], o, -z[..., 0]], -1),
                        torch.stack([-z[..., 1], z[..., 0], o], -1)], -2)


def polar_rotation(M: torch.Tensor) -> torch.Tensor:
    return _PolarRotation.apply(M)


def _cross(a, b):
    return torch.stack([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]])


def _dot(a, b):
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]


def self_targets(prob, x: torch.Tensor, verts: np.ndarray, faces: np.ndarray) -> torch.Tensor:
    """Ray targets c [3, k] of vertices ``verts`` hitting boundary faces ``faces``."""
    start, finc = _incidence(prob)
    fa = prob.faces
    out = []
    for v, f in zip(verts.tolist(), faces.tolist()):
        nv = torch.zeros(3, dtype=x.dtype)
        for g in finc[start[v]:start[v + 1]].tolist():
            i, j, k = fa[g]
            nv = nv + _cross(x[:, j] - x[:, i], x[:, k] - x[:, i])
        d = -nv / torch.sqrt(_dot(nv, nv))
        o = x[:, v]
        a0, a1, a2 = x[:, fa[f, 0]], x[:, fa[f, 1]], x[:, fa[f, 2]]
        e1, e2 = a1 - a0, a2 - a0
        det = _dot(e1, _cross(d, e2))
        t = _dot(e2, _cross(o - a0, e1)) / det
        out.append(o + (t + prob.eps_off) * d)
    return torch.stack(out, dim=1) if out else torch.zeros((3, 0), dtype=x.dtype)


def rhs(prob, x: torch.Tensor, alpha: torch.Tensor, contacts: Contacts, fresh: np.ndarray) -> torch.Tensor:
    """Right-hand side b(x, alpha) [3, n] of the global step with the contact
    set frozen; ``fresh`` [S] marks self contacts whose target follows x."""
    t = tensors(prob)
    p = prob.params
    xe = x[:, prob.tets].permute(2, 0, 1)                     # [T, 3, 4]
    Tt, _ = targets_torch(xe, alpha, t.P, t.Dm_inv, t.vol, t.mode, t.chamber, p.c1, p.c2, p.hyperelastic,
                          rotation=polar_rotation)
    om = torch.from_numpy(prob.omega)
    b = torch.zeros((3, prob.n), dtype=x.dtype)
    for j in range(4):
        b = b.index_add(1, t.tets[j].long(), (om[:, None] * Tt[:, :, j]).T)
    s_idx, slot = np.nonzero(contacts.active)
    if s_idx.size == 0:
        return b
    v = prob.query_verts[s_idx]
    ns = prob.spheres.shape[0]
    eps = prob.eps_off
    c = torch.zeros((3, s_idx.size), dtype=x.dtype)
    xv = x[:, v]
    kept = (slot == 0) & ~np.asarray(fresh, bool)[s_idx]
    new = (slot == 0) & np.asarray(fresh, bool)[s_idx]
    parts = [(np.nonzero(kept)[0], torch.from_numpy(contacts.target[s_idx[kept], 0].T.copy()))]
    if new.any():
        parts.append((np.nonzero(new)[0], self_targets(prob, x, v[new], contacts.prim[s_idx[new], 0])))
    for j in range(ns):
        sel = np.nonzero(slot == 1 + j)[0]
        sph = torch.from_numpy(prob.spheres[j].copy())
        dv = xv[:, sel] - sph[:3, None]
        parts.append((sel, sph[:3, None] + (sph[3] + eps) * dv / torch.sqrt(_dot(dv, dv))))
    for j in range(prob.planes.shape[0]):
        sel = np.nonzero(slot == 1 + ns + j)[0]
        pl = torch.from_numpy(prob.planes[j].copy())
        sd = _dot(pl[3:6, None], xv[:, sel] - pl[:3, None])
        parts.append((sel, xv[:, sel] - (sd - eps) * pl[3:6, None]))
    mo = prob.mesh_obstacle
    if mo is not None:
        sel = np.nonzero(slot == 1 + ns + prob.planes.shape[0])[0]
        if sel.size:
            # closest-point targets on the mesh obstacle: values only (held
            # constant under differentiation; gradients refuse such contacts)
            xn = x.detach().numpy()
            cm = np.stack([mo.target(xn[:, v[i]], eps)[1] for i in sel], axis=1)
            parts.append((sel, torch.from_numpy(cm)))
    for sel, cc in parts:
        c = c.index_copy(1, torch.from_numpy(sel), cc)
    k = torch.from_numpy(prob.k_spring[v])
    return b.index_add(1, torch.from_numpy(v), k * c)


class _Frozen:
    """The frozen-set map's pieces: M_FF factorisation, M_FC x_C."""

    def __init__(self, prob, contacts):
        M, _, _ = system(prob, contacts)
        self.F = np.nonzero(prob.free)[0]
        C = np.nonzero(prob.fixed)[0]
        self.M_FF = M[self.F][:, self.F].tocsc()
        self.lu = spla.splu(self.M_FF)
        self.MxC = (M[self.F][:, C] @ prob.X0[:, C].T).T if C.size else np.zeros((3, self.F.size))


def grad(prob, x, alpha, contacts: Contacts, fresh, dLdx, tol: float = 1e-13, restart: int = 300):
    """dL/dalpha [n_chambers] at positions x [3, n] (a fixed point of the
    frozen-set map) for dL/dx = dLdx [3, n].  Returns (grad, mu [3, n], info).
    Contacts with a triangle-mesh obstacle are not differentiated (refused)."""
    if prob.mesh_obstacle is not None and contacts.active[:, prob.n_slots - 1].any():
        raise NotImplementedError("gradients through triangle-mesh obstacle contacts")
    fz = _Frozen(prob, contacts)
    F, nF = fz.F, fz.F.size
    xt = torch.tensor(np.asarray(x, dtype=np.float64), requires_grad=True)
    at = torch.tensor(np.asarray(alpha, dtype=np.float64).reshape(-1), requires_grad=True)
    b = rhs(prob, xt, at, contacts, np.asarray(fresh, bool))
    g = np.asarray(dLdx, dtype=np.float64)[:, F]

    def vjp(mu_f):
        mu = torch.zeros((3, prob.n), dtype=torch.float64)
        mu[:, F] = torch.from_numpy(mu_f)
        (gx,) = torch.autograd.grad(b, xt, grad_outputs=mu, retain_graph=True)
        return gx.numpy()[:, F]

    def matvec(v):
        mu = v.reshape(3, nF)
        return ((fz.M_FF @ mu.T).T - vjp(mu)).reshape(-1)

    def prec(v):
        return fz.lu.solve(np.ascontiguousarray(v.reshape(3, nF).T)).T.reshape(-1)

    A = spla.LinearOperator((3 * nF, 3 * nF), matvec=matvec, dtype=np.float64)
    P = spla.LinearOperator((3 * nF, 3 * nF), matvec=prec, dtype=np.float64)
    rhs_v = g.reshape(-1)
    mu, code = spla.gmres(A, rhs_v, M=P, rtol=tol, atol=0.0, restart=restart, maxiter=50)
    res = np.linalg.norm(matvec(mu) - rhs_v) / max(np.linalg.norm(rhs_v), 1e-300)
    mu_full = np.zeros((3, prob.n))
    mu_full[:, F] = mu.reshape(3, nF)
    (ga,) = torch.autograd.grad(b, at, grad_outputs=torch.from_numpy(mu_full), retain_graph=False)
    return ga.numpy(), mu_full, dict(gmres=code, residual=res)


def frozen_map(prob, x, alpha, contacts, fresh, fz=None):
    """One global step of the frozen-set map: x -> M_FF^-1 (b_F(x) - M_FC x_C)."""
    fz = fz or _Frozen(prob, contacts)
    with torch.no_grad():
        b = rhs(prob, torch.from_numpy(np.asarray(x, dtype=np.float64)),
                torch.from_numpy(np.asarray(alpha, dtype=np.float64).reshape(-1)), contacts,
                np.asarray(fresh, bool)).numpy()
    xn = np.array(x, dtype=np.float64, copy=True)
    xn[:, fz.F] = fz.lu.solve(np.ascontiguousarray((b[:, fz.F] - fz.MxC).T)).T
    xn[:, prob.fixed] = prob.X0[:, prob.fixed]
    return xn


def frozen_solve(prob, alpha, x0, contacts, fresh, tol: float = 1e-13, max_iter: int = 3000, m: int = 10):
    """Fixed point of the frozen-set map from x0 (Anderson acceleration with
    memory m on the free coordinates).  Stops when max|G(x) - x| <= tol diag.
    Returns (x, iterations, final step)."""
    fz = _Frozen(prob, contacts)
    F = fz.F
    x = np.array(x0, dtype=np.float64, copy=True)
    xs, gs = [], []
    step = np.inf
    for it in range(max_iter):
        gx = frozen_map(prob, x, alpha, contacts, fresh, fz)
        f = (gx - x)[:, F].reshape(-1)
        step = np.abs(f).max() / prob.diag
        if step <= tol:
            return gx, it + 1, step
        xs.append(x[:, F].reshape(-1).copy())
        gs.append(gx[:, F].reshape(-1).copy())
        if len(xs) > m + 1:
            xs.pop(0)
            gs.pop(0)
        if len(xs) == 1:
            x = gx
            continue
        Fm = np.stack([g - xx for g, xx in zip(gs, xs)], axis=1)
        dF = np.diff(Fm, axis=1)
        dG = np.diff(np.stack(gs, axis=1), axis=1)
        gam, *_ = np.linalg.lstsq(dF, Fm[:, -1], rcond=None)
        xf = gs[-1] - dG @ gam
        x = gx.copy()
        x[:, F] = xf.reshape(3, F.size)
    return x, max_iter, step


# ---------------------------------------------------------------------------
# Unrolled gradient over a fixed number of iterations
#
# For K iterations from x_0 the k-th global step is
#     x_{k+1,F} = M_k,FF^-1 (b_k,F(x_k, alpha) - M_k,FC x_C),
# with A_k the contact set the collision check found at x_k (its decisions are
# piecewise constant in x and held as recorded; targets of self contacts
# created at iteration k follow x_k, kept ones are constants, obstacle targets
# follow x_k).  Reverse mode: lambda_K = g, and for k = K-1 ... 0
#     nu = M_k,FF^-1 lambda_{k+1},  dL/dalpha += (db_k/dalpha)^T nu,
#     lambda_k = (db_k/dx_k)^T nu   (free rows).
# The exact global step is the one this definition differentiates; a solver
# whose inner solves are inexact follows a slightly different path.


def record_path(prob, alpha, x0, contacts0, K):
    """K oracle iterations from x0 (and the set contacts0 as A_{-1}), keeping
    (x_k, A_k, fresh_k) for every k and the final x_K."""
    from .collision import collide
    from .local import local_step
    from .solver import _Factor, global_step
    S = prob.query_verts.size
    prev = Contacts.empty(S, prob.n_slots) if contacts0 is None else contacts0.copy()
    x = np.array(x0, dtype=np.float64, copy=True)
    x[:, prob.fixed] = prob.X0[:, prob.fixed]
    fac = _Factor()
    path = []
    for _ in range(K):
        if prob.params.self_collision or prob.params.obstacle_collision:
            A, info = collide(prob, x, prev)
            fresh = info["self_fresh"]
        else:
            A, fresh = Contacts.empty(S, prob.n_slots), np.zeros(S, bool)
        path.append((x.copy(), A, fresh))
        x = global_step(prob, local_step(prob, x, alpha), A, x, fac)
        prev = A
    return path, x


def replay(prob, alpha, path):
    """x_K of the recorded path's contact schedule for another alpha (the
    frozen-schedule map the unrolled gradient differentiates)."""
    x = path[0][0].copy()
    for _, A, fresh in path:
        x = frozen_map(prob, x, alpha, A, fresh)
    return x


def unrolled_grad(prob, alpha, path, dLdx):
    """dL/dalpha and dL/dx_0 of L(x_K) through the recorded path."""
    F = np.nonzero(prob.free)[0]
    lam = np.zeros((3, prob.n))
    lam[:, F] = np.asarray(dLdx, dtype=np.float64)[:, F]
    ga = np.zeros(np.asarray(alpha).size)
    for xk, A, fresh in reversed(path):
        fz = _Frozen(prob, A)
        nu = np.zeros((3, prob.n))
        nu[:, F] = fz.lu.solve(np.ascontiguousarray(lam[:, F].T)).T
        xt = torch.tensor(xk, requires_grad=True)
        at = torch.tensor(np.asarray(alpha, dtype=np.float64).reshape(-1), requires_grad=True)
        b = rhs(prob, xt, at, A, fresh)
        gx, gal = torch.autograd.grad(b, (xt, at), grad_outputs=torch.from_numpy(nu))
        ga += gal.numpy()
        lam = np.zeros((3, prob.n))
        lam[:, F] = gx.numpy()[:, F]
    return ga, lam


def newton_correction(prob, alpha, x, contacts, fresh, rtol: float = 1e-3, maxiter: int = 80, fz=None):
    """One Newton step towards the fixed point of the frozen-set map G near x:
    delta solves (I - G'(x)) delta = G(x) - x on the free coordinates, by
    GMRES with Jacobian-vector products G'(x) v taken as forward differences
    (G(x + s v) - G(x)) / s, s = 1e-7 (1 + max|x|) / max|v| (FP64 map, so
    their error is about 1e-7 relative).  Near a fixed point x + delta is
    that fixed point up to a term of second order in |delta|, so |delta| is
    the distance of x from it.  Returns (delta [3, n], info) with the GMRES
    exit code, its iterations and the map's step max|G(x) - x| / diag."""
    fz = fz or _Frozen(prob, contacts)
    F = fz.F
    x = np.asarray(x, dtype=np.float64)
    gx = frozen_map(prob, x, alpha, contacts, fresh, fz)
    f = (gx - x)[:, F].reshape(-1)
    scale = 1.0 + np.abs(x).max()
    count = [0]

    def matvec(v):
        count[0] += 1
        vm = np.abs(v).max()
        if vm == 0.0:
            return np.zeros_like(v)
        s = 1e-7 * scale / vm
        xv = x.copy()
        xv[:, F] += s * v.reshape(3, F.size)
        gv = frozen_map(prob, xv, alpha, contacts, fresh, fz)
        return v - ((gv - gx)[:, F].reshape(-1)) / s

    A = spla.LinearOperator((f.size, f.size), matvec=matvec, dtype=np.float64)
    d, code = spla.gmres(A, f, rtol=rtol, atol=0.0, restart=maxiter, maxiter=1)
    delta = np.zeros((3, prob.n))
    delta[:, F] = d.reshape(3, F.size)
    return delta, dict(gmres=code, matvecs=count[0], step=float(np.abs(f).max() / prob.diag))
