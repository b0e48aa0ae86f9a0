"""Oracle global step, energy and the local/global iteration (Section III-B).

TEST INFRASTRUCTURE ONLY (see the package docstring).

With the targets T_e, rotations and spring targets fixed by the local step,
Eq. 9 is a least-squares problem in the vertex positions (Section III-B):

    E(x) = sum_e omega_e |x_e N - T_e|_F^2 + sum_{a in A} k_a |x_{v_a} - c_a|^2,

whose minimiser solves M x = b with M = A_el + diag(sum_a k_a e_{v_a}) and
b = sum_e omega_e S_e^T T_e^T + sum_a k_a e_{v_a} c_a^T (T_e is centred, so
T_e N = T_e).  Fixed vertices stay at their rest positions (Dirichlet rows
removed): M[F,F] x_F = b_F - M[F,C] x_C, solved exactly with a sparse direct
factorisation (the paper uses Eigen's direct solvers, Section IV).

Iteration (inner loop of Algorithm 1, readings 13 and 14): from x_0 = X_0 (or
a warm start) and A_{-1} = {} (or an imported set), for k = 0, 1, ...:
collision at x_k with A_{k-1} gives A_k; the local step at x_k gives T_k; the
global step gives x_{k+1}; r_k = max_v |x_{k+1,v} - x_{k,v}| / diag.  Stop
when r_k <= tol and A_k == A_{k-1}, else at max_iter (not converged); with
fixed_iters > 0 run exactly that many iterations.  The paper points to
Anderson acceleration for this fixed-point iteration (end of Section III-B);
``solve(..., anderson=m)`` adds it with an energy safeguard, keeping the
plain iteration's fixed points and stopping rule.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .collision import Contacts, collide
from .local import local_step, gather_elements


def spring_terms(prob, contacts: Contacts | None):
    """Per-vertex spring diagonal d [n] and spring right-hand side [3, n]."""
    d = np.zeros(prob.n)
    bs = np.zeros((3, prob.n))
    if contacts is None or contacts.count == 0:
        return d, bs
    s, slot = np.nonzero(contacts.active)
    v = prob.query_verts[s]
    k = prob.k_spring[v]
    np.add.at(d, v, k)
    for c in range(3):
        np.add.at(bs[c], v, k * contacts.target[s, slot, c])
    return d, bs


def element_rhs(prob, Tt: np.ndarray) -> np.ndarray:
    """sum_e omega_e S_e^T T_e^T as [3, n]."""
    b = np.zeros((3, prob.n))
    w = prob.omega
    for c in range(3):
        for j in range(4):
            b[c] += np.bincount(prob.tets[j], weights=w * Tt[:, c, j], minlength=prob.n)
    return b


def system(prob, contacts):
    d, bs = spring_terms(prob, contacts)
    M = prob.A_el + sp.diags(d)
    return M.tocsr(), d, bs


def residual_rhs(prob, x, Tt, contacts):
    """b - M x on all vertices (zero rows for fixed vertices): the quantity the
    GPU's correction-form solve starts from."""
    M, d, bs = system(prob, contacts)
    r = element_rhs(prob, Tt) + bs - (M @ x.T).T
    r[:, prob.fixed] = 0.0
    return r


class _Factor:
    def __init__(self):
        self.key = None
        self.lu = None


def global_step(prob, Tt, contacts, x_prev, factor: _Factor | None = None):
    """Exact minimiser of Eq. 9 over free vertices; fixed ones stay at X_0."""
    M, d, bs = system(prob, contacts)
    b = element_rhs(prob, Tt) + bs
    F = np.nonzero(prob.free)[0]
    C = np.nonzero(prob.fixed)[0]
    xC = prob.X0[:, C]
    key = d.tobytes()
    if factor is None:
        factor = _Factor()
    if factor.key != key:
        MFF = M[F][:, F].tocsc()
        factor.lu = spla.splu(MFF)
        factor.key = key
    rhs = b[:, F].T - (M[F][:, C] @ xC.T if C.size else 0.0)
    xF = factor.lu.solve(np.ascontiguousarray(rhs))
    x = np.empty((3, prob.n))
    x[:, F] = xF.T
    x[:, C] = xC
    return x


def energy(prob, x, Tt, contacts=None) -> float:
    """Eq. 9 at positions x with the targets held fixed."""
    xe = gather_elements(prob, x)
    D = xe - xe.mean(axis=2, keepdims=True)
    E = float(np.sum(prob.omega * np.sum((D - Tt) ** 2, axis=(1, 2))))
    if contacts is not None and contacts.count:
        s, slot = np.nonzero(contacts.active)
        v = prob.query_verts[s]
        diff = x[:, v].T - contacts.target[s, slot]
        E += float(np.sum(prob.k_spring[v] * np.sum(diff * diff, axis=1)))
    return E


def step(prob, x, alpha, prev: Contacts | None, factor=None):
    """One local/global iteration from x_k with A_{k-1} = prev.

    Returns (x_{k+1}, A_k, T_k, info) where info has r_k, E_k (energy of x_k
    with the new targets), E_sur (energy of x_{k+1} with the same targets) and
    the collision diagnostics.
    """
    S = prob.query_verts.size
    if prev is None:
        prev = Contacts.empty(S, prob.n_slots)
    if prob.params.self_collision or prob.params.obstacle_collision:
        A, cinfo = collide(prob, x, prev)
    else:
        A, cinfo = Contacts.empty(S, prob.n_slots), dict(ray_miss=0)
    Tt = local_step(prob, x, alpha)
    xn = global_step(prob, Tt, A, x, factor)
    dx = xn - x
    r = float(np.max(np.sqrt((dx[0] * dx[0] + dx[1] * dx[1]) + dx[2] * dx[2]))) / prob.diag
    info = dict(r=r, E=energy(prob, x, Tt, A), E_sur=energy(prob, xn, Tt, A),
                ray_miss=cinfo.get("ray_miss", 0), changed=not A.same_set(prev),
                n_contacts=A.count)
    return xn, A, Tt, info


def anderson_update(g, f, dX, dF):
    """One Anderson (type II) update of a fixed-point iteration x -> G(x)
    (Walker & Ni 2011): with the current residual f = G(x) - x, the image
    g = G(x) and the last differences dX_j = x_{j+1} - x_j, dF_j = f_{j+1} - f_j
    as the columns of dX and dF,

        gamma = argmin_gamma |f - dF gamma|_2,   x_new = g - (dX + dF) gamma

    (dX + dF holds the differences of G).  With no columns it is the plain step
    x_new = g.  The least-squares problem is solved by numpy's lstsq."""
    if dF.shape[1] == 0:
        return g.copy(), np.zeros(0)
    gam, *_ = np.linalg.lstsq(dF, f, rcond=None)
    return g - (dX + dF) @ gam, gam


def solve(prob, alpha, x0=None, contacts0: Contacts | None = None, max_iter=None,
          fixed_iters=None, tol=None, history: bool = False, callback=None, anderson: int = 0,
          aa_guard: str = "residual", aa_slack: float = 0.5, aa_keep_set: bool = True):
    """Local/global iteration to convergence (or a fixed iteration count).

    With ``anderson`` = m > 0 the iteration is Anderson-accelerated (memory m)
    with a safeguard, after Peng et al. (2018) for local/global solvers; the
    fixed points, and the stopping rule, are those of the plain iteration.
    Every iteration evaluates the plain map at the current point x_k
    (collision, local step, exact global step: G(x_k)), its residual and its
    energy E_k (Eq. 9 at x_k with the targets and contact set found there):

    * r_k = max_v |G(x_k)_v - x_k,v| / diag; converged (result G(x_k)) when
      r_k <= tol and the active set is unchanged, as in the plain iteration;
    * x_k was an accelerated point and fails the guard: with
      aa_guard = "residual", r_k > (1 + aa_slack) r_acc; with "energy",
      E_k > E_acc + aa_slack |E_acc| (r_acc, E_acc: those of the last
      accepted point); "none" has no value test; with aa_keep_set an
      accelerated x_k whose active set differs from the last accepted
      point's is rejected too.  A rejected x_k is replaced by the plain step
      G(x_acc) from the last accepted point, evaluated with that point's
      active set as the previous one (the plain iteration's state), and the
      history is cleared;
    * otherwise x_k is accepted (E_acc = E_k): the history gains
      (x_k - x_prev, f_k - f_prev) with f = G(x) - x (after being cleared
      when the active set changed), keeps its last m columns, and the next
      point is ``anderson_update`` of G(x_k).

    The last iteration (fixed_iters or max_iter reached) ends on the plain
    step G(x_k), as a converged one does.  Fixed vertices stay at their rest
    positions (their differences are zero).  Returns (x, contacts, stats) with stats = dict(iters, residual,
    converged, n_contacts, ray_miss, energy, history, rejected).
    """
    p = prob.params
    max_iter = p.max_iter if max_iter is None else max_iter
    fixed_iters = p.fixed_iters if fixed_iters is None else fixed_iters
    tol = p.tol if tol is None else tol
    x = prob.X0.copy() if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    x[:, prob.fixed] = prob.X0[:, prob.fixed]
    S = prob.query_verts.size
    prev = Contacts.empty(S, prob.n_slots) if contacts0 is None else contacts0.copy()
    factor = _Factor()
    hist = []
    n_it = fixed_iters if fixed_iters > 0 else max_iter
    converged = False
    info = dict(r=np.inf, E=np.nan, ray_miss=0, n_contacts=0)
    m = int(anderson)
    if aa_guard not in ("residual", "energy", "none"):
        raise ValueError("aa_guard must be 'residual', 'energy' or 'none'")
    cand = False                   # x is an accelerated point (not yet accepted)
    e_acc = np.inf                 # energy of the last accepted point
    r_acc = np.inf                 # residual of the last accepted point
    x_fb = None                    # plain step from the last accepted point
    x_prev = f_prev = None         # last accepted point and its residual
    A_acc = None                   # active set found at the last accepted point
    dX, dF = [], []
    rejected = 0
    k = 0
    for k in range(n_it):
        xn, A, Tt, info = step(prob, x, alpha, prev, factor)
        if history:
            hist.append(dict(k=k, E=info["E"], E_sur=info["E_sur"], r=info["r"],
                             n_contacts=info["n_contacts"], changed=info["changed"], cand=cand))
        if callback is not None:
            callback(k, x, xn, A, info)
        done = info["r"] <= tol and not info["changed"]
        prev = A
        if history:
            hist[-1]["accepted"] = True
        stop = fixed_iters <= 0 and done
        if m <= 0 or stop:
            x = xn
            if stop:
                converged = True
                break
            continue
        reject = cand and ((aa_guard == "residual" and not info["r"] <= (1.0 + aa_slack) * r_acc) or
                           (aa_guard == "energy" and not info["E"] <= e_acc + aa_slack * abs(e_acc)) or
                           (aa_keep_set and info["changed"]))
        if reject:
            rejected += 1
            if history:
                hist[-1]["accepted"] = False
        if k == n_it - 1:
            x = xn                 # the last iteration ends on the plain step
            break
        if reject:
            x = x_fb
            prev = A_acc.copy()
            cand = False
            x_prev = f_prev = None
            dX, dF = [], []
            continue
        e_acc, r_acc = info["E"], info["r"]
        A_acc = A.copy()
        f = xn - x
        if info["changed"]:
            x_prev = f_prev = None
            dX, dF = [], []
        if x_prev is not None:
            dX.append((x - x_prev).reshape(-1))
            dF.append((f - f_prev).reshape(-1))
            if len(dX) > m:
                dX.pop(0)
                dF.pop(0)
        x_prev, f_prev = x.copy(), f.copy()
        x_fb = xn
        if dX:
            xa, _ = anderson_update(xn.reshape(-1), f.reshape(-1), np.stack(dX, axis=1), np.stack(dF, axis=1))
            x = xa.reshape(3, -1)
            cand = True
        else:
            x = xn
            cand = False
    if fixed_iters > 0:
        converged = info["r"] <= tol and not info["changed"]
    stats = dict(iters=(k + 1) if n_it > 0 else 0, residual=info["r"], converged=converged,
                 n_contacts=prev.count, ray_miss=info["ray_miss"], energy=info["E"],
                 history=hist, rejected=rejected)
    return x, prev, stats
