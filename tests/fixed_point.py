"""Parity of a converged GPU result with the oracle's fixed point (test helper).

The local/global iteration with collision response has many fixed points
(hysteresis of the active set), so a converged GPU result is checked against
the oracle's fixed point for the GPU's own final active set: the oracle's
frozen-set map (the plain map with that contact set held, new self-contact
targets following x) is iterated from the GPU result to a 1e-11 step, then
the oracle's collision check at that point, with the GPU set as the previous
one, must return the same set.  The distance between the two points is the
parity error."""
import numpy as np

import oracle
from oracle import adjoint as oa
from oracle.collision import Contacts


def oracle_contacts(prob, cg, lo=0):
    """The oracle's dense contact set (and fresh flags per query vertex) from a
    GPU listing (rows (v, type, prim), target, normal, fresh) of vertices
    offset by lo."""
    A = Contacts.empty(prob.query_verts.size, prob.n_slots)
    fresh = np.zeros(prob.query_verts.size, bool)
    ns, npl = prob.spheres.shape[0], prob.planes.shape[0]
    for i, ((v, typ, prim), t, nrm) in enumerate(zip(cg["rows"], cg["target"], cg["normal"])):
        s = int(np.searchsorted(prob.query_verts, v - lo))
        sl = 0 if typ == 0 else (1 + prim if typ == 1 else (1 + ns + prim if typ == 2 else 1 + ns + npl))
        A.active[s, sl] = True
        A.target[s, sl], A.normal[s, sl], A.prim[s, sl] = t, nrm, prim
        if typ == 0 and "fresh" in cg and cg["fresh"][i]:
            fresh[s] = True
    return A, fresh


def check(prob, alpha, xg, cg, lo=0, tol=1e-11, max_iter=4000, broadphase="brute"):
    """Returns dict(err (max distance / diag), same_set, iters, step, x) for
    the GPU result xg [3, n] (float64) with listing cg."""
    A, fresh = oracle_contacts(prob, cg, lo)
    xo, its, step = oa.frozen_solve(prob, alpha, np.asarray(xg, dtype=np.float64), A, fresh, tol=tol,
                                    max_iter=max_iter)
    A2, info = oracle.collide(prob, xo, A, broadphase=broadphase)
    same = (A2.same_set(A) and np.array_equal(A2.prim[A.active], A.prim[A.active])
            and np.array_equal(info["self_fresh"], fresh))
    err = float(np.abs(np.asarray(xg, dtype=np.float64) - xo).max() / prob.diag)
    return dict(err=err, same_set=bool(same), iters=its, step=step, x=xo, contacts=A.count)
