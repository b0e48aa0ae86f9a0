"""Oracle local step: per-element target shapes (Section III-A).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Written in plain PyTorch (CPU, float64) so that the same definition serves
the forward solve and, through automatic differentiation, the gradient
oracle.  For an element with current positions x_e (3x4), D = x_e N is its
centred current shape and P = X_e N its centred rest shape.

Chamber element (Section III-A.1).  The target scales the rest shape so that
the element volume becomes alpha times its rest volume: Q = alpha^(1/3) P for
an isotropic chamber, Q = diag(s) P with s_axis = alpha (other entries 1) for
an axis-actuated one (length actuation, footnote of Section II-A; reading 8).
The rotation R aligning Q with D is the Kabsch fit from the SVD of D Q^T
(below Eq. 1), and the target is T = R Q.

Body element (Section III-A.2).  R is the Kabsch fit of P to D.  The blend of
Eq. 6, B = (1 - w) D + w R P, is written in the current frame (the paper's
rest-frame form rotated by R, reading 2).  The weight w = R_w(lambda) is the
Mooney-Rivlin secant-stiffness ratio (reading 4; the paper defers its form to
its reference [Christ21]):

    w(lambda) = (1 + 1/lambda + 1/lambda^2) (c1 + c2/lambda) / (3 (c1 + c2)),

the uniaxial nominal stress 2 (lambda - lambda^-2)(c1 + c2/lambda) over its
linearisation 6 (c1 + c2)(lambda - 1), with the effective stretch
lambda = sqrt(Ibar1 / 3), Ibar1 = J^(-2/3) |F|_F^2, F = Ds Dm^-1 (lambda = 1
when J <= 0).  Eq. 7 is circular as printed; its stated purpose (keep the
element volume, "incompressibility") fixes the reading
T = (Vol(e) / Vol(B))^(1/3) B (reading 3); an inverted B (Vol(B) <= 0) falls
back to T = R P.
"""
from __future__ import annotations

import numpy as np
import torch

from .mesh import BODY, CH_ISO, CH_AX_X, CH_AX_Y, CH_AX_Z, centring


def mooney_rivlin_weight(lam, c1: float, c2: float):
    """R_w(lambda): secant over initial stiffness of uniaxial Mooney-Rivlin."""
    il = 1.0 / lam
    return (1.0 + il + il * il) * (c1 + c2 * il) / (3.0 * (c1 + c2))


def kabsch(M: torch.Tensor) -> torch.Tensor:
    """Rotation R maximising tr(R^T M): R = U diag(1,1,d) W^T with M = U S W^T
    and d = sign det(U W^T) (sign 0 counts as +1)."""
    U, _, Vh = torch.linalg.svd(M)
    d = torch.sign(torch.linalg.det(U) * torch.linalg.det(Vh))
    d = torch.where(d == 0, torch.ones_like(d), d)
    ones = torch.ones_like(d)
    Dg = torch.diag_embed(torch.stack([ones, ones, d], dim=-1))
    return U @ Dg @ Vh


def _det3(A: torch.Tensor) -> torch.Tensor:
    return torch.linalg.det(A)


def targets_torch(xe: torch.Tensor, alpha: torch.Tensor, P: torch.Tensor, Dm_inv: torch.Tensor,
                  vol: torch.Tensor, mode: torch.Tensor, chamber: torch.Tensor,
                  c1: float, c2: float, hyperelastic: bool, rotation=None):
    """Target shapes T_e (T,3,4) and rotations R_e for current positions xe (T,3,4).

    Differentiable in xe and alpha (float64 tensors).  ``rotation`` replaces
    ``kabsch`` (same values; the gradient oracle passes one with an explicit
    derivative).
    """
    Nm = torch.as_tensor(centring(), dtype=xe.dtype)
    D = xe @ Nm
    is_ch = mode != BODY
    ch = torch.clamp(chamber, min=0)
    a = alpha[ch]                                              # per-tet alpha (body: unused)
    one = torch.ones_like(a)
    s_iso = torch.pow(a, 1.0 / 3.0)
    sx = torch.where(mode == CH_ISO, s_iso, torch.where(mode == CH_AX_X, a, one))
    sy = torch.where(mode == CH_ISO, s_iso, torch.where(mode == CH_AX_Y, a, one))
    sz = torch.where(mode == CH_ISO, s_iso, torch.where(mode == CH_AX_Z, a, one))
    S = torch.stack([sx, sy, sz], dim=-1)
    S = torch.where(is_ch[:, None], S, torch.ones_like(S))
    Q = S[:, :, None] * P                                      # diag(s) P; body: P
    R = (rotation or kabsch)(D @ Q.transpose(1, 2))
    RQ = R @ Q

    # body blend (Eq. 6) and volume scaling (Eq. 7)
    Ds = xe[:, :, 1:] - xe[:, :, :1]
    F = Ds @ Dm_inv
    J = _det3(F)
    I1 = (F * F).sum(dim=(1, 2))
    Jsafe = torch.where(J > 0, J, torch.ones_like(J))
    lam = torch.where(J > 0, torch.sqrt(torch.pow(Jsafe, -2.0 / 3.0) * I1 / 3.0), torch.ones_like(J))
    if hyperelastic:
        w = mooney_rivlin_weight(lam, c1, c2)
    else:
        w = torch.ones_like(lam)
    B = (1.0 - w)[:, None, None] * D + w[:, None, None] * RQ
    VB = _det3(B[:, :, 1:] - B[:, :, :1]) / 6.0
    VBsafe = torch.where(VB > 0, VB, torch.ones_like(VB))
    scale = torch.pow(vol / VBsafe, 1.0 / 3.0)
    Tbody = torch.where((VB > 0)[:, None, None], scale[:, None, None] * B, RQ)
    Tt = torch.where(is_ch[:, None, None], RQ, Tbody)
    return Tt, dict(R=R, D=D, w=w, lam=lam, VB=VB, J=J)


class _Tensors:
    """Torch views of a Problem's rest data (built once per Problem)."""

    def __init__(self, prob):
        self.P = torch.from_numpy(prob.P)
        self.Dm_inv = torch.from_numpy(prob.Dm_inv)
        self.vol = torch.from_numpy(prob.vol)
        self.mode = torch.from_numpy(prob.mode)
        self.chamber = torch.from_numpy(prob.chamber)
        self.tets = torch.from_numpy(prob.tets)


def tensors(prob) -> _Tensors:
    t = getattr(prob, "_torch", None)
    if t is None:
        t = _Tensors(prob)
        prob._torch = t
    return t


def gather_elements(prob, x: np.ndarray) -> np.ndarray:
    """x_e for every tet: [T, 3, 4] from x [3, n]."""
    return np.moveaxis(x[:, prob.tets], 2, 0)


def local_step(prob, x: np.ndarray, alpha, aux: bool = False):
    """Target shapes T_e [T,3,4] (numpy, FP64) at positions x [3,n]."""
    t = tensors(prob)
    xe = torch.from_numpy(np.ascontiguousarray(gather_elements(prob, np.asarray(x, dtype=np.float64))))
    al = torch.as_tensor(np.asarray(alpha, dtype=np.float64).reshape(-1))
    p = prob.params
    with torch.no_grad():
        Tt, extra = targets_torch(xe, al, t.P, t.Dm_inv, t.vol, t.mode, t.chamber,
                                  p.c1, p.c2, p.hyperelastic)
    if aux:
        return Tt.numpy(), {k: v.numpy() for k, v in extra.items()}
    return Tt.numpy()
