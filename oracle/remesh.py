"""Oracle: the remesh checks and the progressive actuation of Algorithm 1's
outer loop (Section III-B).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper raises the actuation in stages and, after each stage, asks for the
chamber region to be remeshed when one of its elements either grew in volume
by more than alpha_max, or carries a distortion norm(Sigma) above d_max, where
Sigma holds the singular values of the affine map taking the deformed element
onto its undeformed one (alpha_max = d_max = 4).  Remeshing itself is a host
tool and not part of this oracle; what is computed here is the decision.

Readings (the paper leaves these open):

* reference shape: the element as it was last meshed.  Without a remesher
  that is the rest shape; a caller may pass any other reference (e.g. the
  previous stage's positions).  The volume test of Section III-B (against the
  undeformed element) and that of Algorithm 1 (against the previous stage)
  coincide when every flagged stage is followed by a remesh;
* the affine map taking the deformed element to the reference one is the
  inverse of the deformation gradient F = D_x D_ref^-1 (D: the three edge
  vectors from the first vertex), so its singular values are 1/sigma_i(F);
* norm(Sigma) is the 2-norm of the diagonal Sigma, its largest entry:
  norm(Sigma) = 1 / sigma_min(F).  The test therefore fires when some
  direction of the element was squashed below 1/d_max of its length (a
  singular or inverted-to-flat element fires it; 1/0 is infinite);
* only chamber elements (M_c) are checked; body elements never flag;
* the volume ratio is det(D_x) / det(D_ref) (signed: an inverted chamber
  element does not pass the volume test, its distortion test decides);
* stages: alpha_k = min(alpha, (k+1) alpha_max) per chamber, k = 0, 1, ...,
  until every chamber has its target (Algorithm 1 starts at alpha_max and adds
  alpha_max per stage; capping at the target avoids overshooting it).  Each
  stage is a complete solve warm-started from the previous stage's positions
  and active contact set.

Flags are one byte per tet: bit 0 (VOLUME) and bit 1 (DISTORTION).  Both
decisions are taken in FP64.
"""
from __future__ import annotations

import numpy as np

from .mesh import BODY
from .solver import solve

VOLUME, DISTORTION = 1, 2


def edge_matrices(prob, pos) -> np.ndarray:
    """[T, 3, 3]: columns are the edges v1-v0, v2-v0, v3-v0 of each tet
    (in the oracle's oriented vertex order) at positions ``pos`` [3, n]."""
    pe = np.moveaxis(np.asarray(pos, dtype=np.float64)[:, prob.tets], 2, 0)   # [T, 3, 4]
    return pe[:, :, 1:] - pe[:, :, :1]


def remesh_measures(prob, x, x_ref=None):
    """Per tet: volume ratio Vol(x_e) / Vol(ref_e) and norm(Sigma) = 1/sigma_min(F)
    (both FP64; infinite where F is singular)."""
    ref = prob.X0 if x_ref is None else x_ref
    Dx, Dr = edge_matrices(prob, x), edge_matrices(prob, ref)
    ratio = np.linalg.det(Dx) / np.linalg.det(Dr)
    F = Dx @ np.linalg.inv(Dr)
    smin = np.linalg.svd(F, compute_uv=False)[:, -1]
    with np.errstate(divide="ignore"):
        dist = 1.0 / smin
    return ratio, dist


def remesh_flags(prob, x, x_ref=None, alpha_max: float = 4.0, d_max: float = 4.0) -> np.ndarray:
    """uint8 [T]: VOLUME where ratio > alpha_max, DISTORTION where
    norm(Sigma) > d_max, for chamber elements; 0 for body elements."""
    ratio, dist = remesh_measures(prob, x, x_ref)
    chamber = prob.mode != BODY
    f = np.where(chamber & (ratio > alpha_max), VOLUME, 0) | np.where(chamber & (dist > d_max), DISTORTION, 0)
    return f.astype(np.uint8)


def stage_alphas(alpha, alpha_max: float = 4.0) -> list[np.ndarray]:
    """The actuation of every stage: alpha_k = min(alpha, (k+1) alpha_max)
    until alpha_k = alpha for every chamber (one stage when alpha <= alpha_max)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    if not (np.all(np.isfinite(alpha)) and np.isfinite(alpha_max) and alpha_max > 0):
        raise ValueError("alpha and alpha_max must be finite, alpha_max > 0")
    out, k = [], 0
    while True:
        ak = np.minimum(alpha, (k + 1) * alpha_max)
        out.append(ak)
        if np.all(ak >= alpha):
            return out
        k += 1


def solve_progressive(prob, alpha, alpha_max: float = 4.0, d_max: float = 4.0, stop_on_flag: bool = True,
                      x0=None, contacts0=None, **solve_kw):
    """Algorithm 1's outer loop without the remesher: solve each stage, then
    take the remesh decision at its result (against the rest shape).  With
    ``stop_on_flag`` the loop ends after the first stage that flags an
    element (the caller would remesh there and continue on the new mesh).
    Returns (x, contacts, flags, stages) with stages a list of
    dict(alpha, stats, n_flagged)."""
    x, prev = x0, contacts0
    stages, flags = [], np.zeros(prob.T, dtype=np.uint8)
    for ak in stage_alphas(alpha, alpha_max):
        x, prev, st = solve(prob, ak, x0=x, contacts0=prev, **solve_kw)
        flags = remesh_flags(prob, x, None, alpha_max, d_max)
        nf = int(np.count_nonzero(flags))
        stages.append(dict(alpha=ak, stats=st, n_flagged=nf))
        if stop_on_flag and nf > 0:
            break
    return x, prev, flags, stages
