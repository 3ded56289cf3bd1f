"""Lie groups SE(2) and SE(3) for the oracle (PyTorch CPU, float64).

The paper computes exponential and logarithm maps, inverse and composition
in closed form and differentiates on the tangent space with right
perturbations g*tau(s*xi) (Section 3 "Differentiable Lie groups",
Appendix D, Eq. grad1).  This module writes those maps from their
definitions:

* elements are homogeneous matrices ([...,3,3] for SE(2), [...,4,4] for SE(3));
* tangents are ordered [translation; rotation]: xi = (rho_x, rho_y, theta)
  for SE(2) and xi = (rho, phi) in R^6 for SE(3);
* hat(xi) is the Lie-algebra matrix, exp uses the Rodrigues / V(phi) closed
  form, log inverts it (V^-1 applied with a linear solve);
* ad(xi) is the matrix of the Lie bracket [xi, .] and Ad(X) the adjoint;
* the right Jacobian is taken from its series definition
  Jr(xi) = sum_n (-ad xi)^n / (n+1)!, summed until the terms vanish, and
  Jr^-1 is its matrix inverse.

All functions broadcast over leading dimensions and are differentiable with
torch.autograd (the small-angle branches use the "double where" pattern so
that no NaN gradient leaks from the unused branch).
"""
from __future__ import annotations

import math

import torch

DT = torch.float64
_SMALL = 1e-4  # below this angle the Taylor forms are exact to rounding in float64
_SERIES_TERMS = 48


def _t(x) -> torch.Tensor:
    return torch.as_tensor(x, dtype=DT)


# ---------------------------------------------------------------------------
# SO(3)
# ---------------------------------------------------------------------------
def so3_hat(w: torch.Tensor) -> torch.Tensor:
    z = torch.zeros_like(w[..., 0])
    return torch.stack([
        torch.stack([z, -w[..., 2], w[..., 1]], -1),
        torch.stack([w[..., 2], z, -w[..., 0]], -1),
        torch.stack([-w[..., 1], w[..., 0], z], -1),
    ], -2)


def so3_vee(W: torch.Tensor) -> torch.Tensor:
    return torch.stack([W[..., 2, 1], W[..., 0, 2], W[..., 1, 0]], -1)


def _sinc_coeffs(th2: torch.Tensor):
    """A = sin(t)/t, B = (1-cos t)/t^2, C = (t - sin t)/t^3 as functions of t^2."""
    small = th2 < _SMALL ** 2
    safe = torch.where(small, torch.ones_like(th2), th2)
    t = torch.sqrt(safe)
    A = torch.where(small, 1 - th2 / 6 + th2 ** 2 / 120, torch.sin(t) / t)
    B = torch.where(small, 0.5 - th2 / 24 + th2 ** 2 / 720, (1 - torch.cos(t)) / safe)
    C = torch.where(small, 1.0 / 6 - th2 / 120 + th2 ** 2 / 5040, (t - torch.sin(t)) / (safe * t))
    return A, B, C


def so3_exp(w: torch.Tensor) -> torch.Tensor:
    th2 = (w * w).sum(-1)
    A, B, _ = _sinc_coeffs(th2)
    W = so3_hat(w)
    I = torch.eye(3, dtype=DT).expand(W.shape)
    return I + A[..., None, None] * W + B[..., None, None] * (W @ W)


def so3_log(R: torch.Tensor) -> torch.Tensor:
    """Rotation vector of R; angle from atan2(|axis*sin|, cos), the axis taken
    from the symmetric part of R when the angle approaches pi."""
    w = 0.5 * so3_vee(R - R.transpose(-1, -2))          # sin(t) * axis
    cos_t = 0.5 * (R.diagonal(dim1=-2, dim2=-1).sum(-1) - 1.0)
    s2 = (w * w).sum(-1)
    small = (s2 < _SMALL ** 2) & (cos_t > 0)               # angle near 0: series in sin^2
    pos = s2 > 0
    s_abs = torch.where(pos, torch.sqrt(torch.where(pos, s2, torch.ones_like(s2))), torch.zeros_like(s2))
    theta = torch.atan2(s_abs, cos_t)
    fac_small = 1 + s2 / 6 + 3 * s2 * s2 / 40           # t/sin t as a series in sin^2 t
    denom = torch.where(small | ~pos, torch.ones_like(s_abs), s_abs)
    fac = torch.where(small, fac_small, theta / denom)
    phi_reg = fac[..., None] * w
    # near pi: (R + R^T)/2 - cos(t) I = (1 - cos t) a a^T
    near_pi = cos_t < -0.9
    Bm = 0.5 * (R + R.transpose(-1, -2)) - cos_t[..., None, None] * torch.eye(3, dtype=DT)
    one_m_cos = torch.where(near_pi, 1 - cos_t, torch.ones_like(cos_t))
    aat = Bm / one_m_cos[..., None, None]
    diag = aat.diagonal(dim1=-2, dim2=-1)
    k = diag.argmax(-1)
    col = torch.gather(aat, -1, k[..., None, None].expand(*aat.shape[:-1], 1))[..., 0]
    dk = torch.gather(diag, -1, k[..., None])[..., 0]
    axis = col / torch.sqrt(torch.where(near_pi, dk, torch.ones_like(dk)))[..., None]
    sgn = torch.where((axis * w).sum(-1) < 0, -torch.ones_like(dk), torch.ones_like(dk))
    phi_pi = (sgn * theta)[..., None] * axis
    return torch.where(near_pi[..., None], phi_pi, phi_reg)


# ---------------------------------------------------------------------------
# SE(3): xi = (rho, phi)
# ---------------------------------------------------------------------------
def se3_from34(T34: torch.Tensor) -> torch.Tensor:
    T34 = _t(T34)
    bottom = torch.zeros(*T34.shape[:-2], 1, 4, dtype=DT)
    bottom[..., 0, 3] = 1.0
    return torch.cat([T34, bottom], -2)


def se3_to34(T: torch.Tensor) -> torch.Tensor:
    return T[..., :3, :]


def se3_hat(xi: torch.Tensor) -> torch.Tensor:
    top = torch.cat([so3_hat(xi[..., 3:]), xi[..., :3, None]], -1)
    bottom = torch.zeros(*xi.shape[:-1], 1, 4, dtype=DT)
    return torch.cat([top, bottom], -2)


def se3_vee(M: torch.Tensor) -> torch.Tensor:
    return torch.cat([M[..., :3, 3], so3_vee(M[..., :3, :3])], -1)


def so3_V(phi: torch.Tensor) -> torch.Tensor:
    th2 = (phi * phi).sum(-1)
    _, B, C = _sinc_coeffs(th2)
    W = so3_hat(phi)
    I = torch.eye(3, dtype=DT).expand(W.shape)
    return I + B[..., None, None] * W + C[..., None, None] * (W @ W)


def se3_exp(xi: torch.Tensor) -> torch.Tensor:
    R = so3_exp(xi[..., 3:])
    t = (so3_V(xi[..., 3:]) @ xi[..., :3, None])[..., 0]
    top = torch.cat([R, t[..., None]], -1)
    bottom = torch.zeros(*xi.shape[:-1], 1, 4, dtype=DT)
    bottom[..., 0, 3] = 1.0
    return torch.cat([top, bottom], -2)


def se3_log(T: torch.Tensor) -> torch.Tensor:
    phi = so3_log(T[..., :3, :3])
    rho = torch.linalg.solve(so3_V(phi), T[..., :3, 3:4])[..., 0]
    return torch.cat([rho, phi], -1)


def se3_inv(T: torch.Tensor) -> torch.Tensor:
    R = T[..., :3, :3]
    Rt = R.transpose(-1, -2)
    t = -(Rt @ T[..., :3, 3:4])
    top = torch.cat([Rt, t], -1)
    return torch.cat([top, T[..., 3:4, :]], -2)


def se3_ad(xi: torch.Tensor) -> torch.Tensor:
    """Matrix of [xi, .] on (rho, phi) tangents: [[phi^, rho^], [0, phi^]]."""
    P = so3_hat(xi[..., 3:])
    Rh = so3_hat(xi[..., :3])
    Z = torch.zeros_like(P)
    return torch.cat([torch.cat([P, Rh], -1), torch.cat([Z, P], -1)], -2)


def se3_Ad(T: torch.Tensor) -> torch.Tensor:
    """Adjoint: X exp(xi) X^-1 = exp(Ad_X xi); [[R, t^ R], [0, R]]."""
    R = T[..., :3, :3]
    tR = so3_hat(T[..., :3, 3]) @ R
    Z = torch.zeros_like(R)
    return torch.cat([torch.cat([R, tR], -1), torch.cat([Z, R], -1)], -2)


# ---------------------------------------------------------------------------
# SE(2): elements 3x3, xi = (rho_x, rho_y, theta)
# ---------------------------------------------------------------------------
def se2_from4(p: torch.Tensor) -> torch.Tensor:
    """(x, y, cos, sin) -> 3x3 homogeneous matrix."""
    p = _t(p)
    x, y, c, s = p[..., 0], p[..., 1], p[..., 2], p[..., 3]
    z, o = torch.zeros_like(x), torch.ones_like(x)
    return torch.stack([torch.stack([c, -s, x], -1), torch.stack([s, c, y], -1),
                        torch.stack([z, z, o], -1)], -2)


def se2_to4(T: torch.Tensor) -> torch.Tensor:
    return torch.stack([T[..., 0, 2], T[..., 1, 2], T[..., 0, 0], T[..., 1, 0]], -1)


def se2_hat(xi: torch.Tensor) -> torch.Tensor:
    z = torch.zeros_like(xi[..., 0])
    th = xi[..., 2]
    return torch.stack([torch.stack([z, -th, xi[..., 0]], -1), torch.stack([th, z, xi[..., 1]], -1),
                        torch.stack([z, z, z], -1)], -2)


def se2_vee(M: torch.Tensor) -> torch.Tensor:
    return torch.stack([M[..., 0, 2], M[..., 1, 2], M[..., 1, 0]], -1)


def _so2_V(th: torch.Tensor) -> torch.Tensor:
    A, B, _ = _sinc_coeffs(th * th)          # sin t / t, (1 - cos t)/t^2
    Bt = B * th                              # (1 - cos t)/t
    return torch.stack([torch.stack([A, -Bt], -1), torch.stack([Bt, A], -1)], -2)


def se2_exp(xi: torch.Tensor) -> torch.Tensor:
    th = xi[..., 2]
    c, s = torch.cos(th), torch.sin(th)
    t = (_so2_V(th) @ xi[..., :2, None])[..., 0]
    z, o = torch.zeros_like(th), torch.ones_like(th)
    return torch.stack([torch.stack([c, -s, t[..., 0]], -1), torch.stack([s, c, t[..., 1]], -1),
                        torch.stack([z, z, o], -1)], -2)


def se2_log(T: torch.Tensor) -> torch.Tensor:
    th = torch.atan2(T[..., 1, 0], T[..., 0, 0])
    rho = torch.linalg.solve(_so2_V(th), T[..., :2, 2:3])[..., 0]
    return torch.cat([rho, th[..., None]], -1)


def se2_inv(T: torch.Tensor) -> torch.Tensor:
    R = T[..., :2, :2]
    Rt = R.transpose(-1, -2)
    t = -(Rt @ T[..., :2, 2:3])
    return torch.cat([torch.cat([Rt, t], -1), T[..., 2:3, :]], -2)


def se2_ad(xi: torch.Tensor) -> torch.Tensor:
    """Matrix of [xi, .]: [[0, -th, rho_y], [th, 0, -rho_x], [0, 0, 0]]."""
    z = torch.zeros_like(xi[..., 0])
    th = xi[..., 2]
    return torch.stack([torch.stack([z, -th, xi[..., 1]], -1), torch.stack([th, z, -xi[..., 0]], -1),
                        torch.stack([z, z, z], -1)], -2)


def se2_Ad(T: torch.Tensor) -> torch.Tensor:
    """Adjoint: [[R, (t_y, -t_x)^T], [0, 1]]."""
    c, s = T[..., 0, 0], T[..., 1, 0]
    x, y = T[..., 0, 2], T[..., 1, 2]
    z, o = torch.zeros_like(c), torch.ones_like(c)
    return torch.stack([torch.stack([c, -s, y], -1), torch.stack([s, c, -x], -1),
                        torch.stack([z, z, o], -1)], -2)


# ---------------------------------------------------------------------------
# right Jacobian from its series definition
# ---------------------------------------------------------------------------
def right_jacobian(ad: torch.Tensor) -> torch.Tensor:
    """Jr = sum_{n>=0} (-ad)^n / (n+1)!  (ad = matrix of the bracket with xi)."""
    d = ad.shape[-1]
    I = torch.eye(d, dtype=DT).expand(ad.shape)
    M = -ad
    term = I.clone()
    out = I.clone()
    for n in range(1, _SERIES_TERMS):
        term = term @ M / (n + 1)
        out = out + term
    return out


class Group:
    """Bundle of the maps of one group so costs can be written once."""

    def __init__(self, name: str):
        self.name = name
        if name == "SE3":
            self.dof, self.mat = 6, 4
            self.exp, self.log, self.inv = se3_exp, se3_log, se3_inv
            self.ad, self.Ad, self.hat, self.vee = se3_ad, se3_Ad, se3_hat, se3_vee
            self.from_storage, self.to_storage = se3_from34, se3_to34
        elif name == "SE2":
            self.dof, self.mat = 3, 3
            self.exp, self.log, self.inv = se2_exp, se2_log, se2_inv
            self.ad, self.Ad, self.hat, self.vee = se2_ad, se2_Ad, se2_hat, se2_vee
            self.from_storage, self.to_storage = se2_from4, se2_to4
        else:
            raise ValueError(name)

    def jr(self, xi: torch.Tensor) -> torch.Tensor:
        return right_jacobian(self.ad(xi))

    def jr_inv(self, xi: torch.Tensor) -> torch.Tensor:
        return torch.linalg.inv(self.jr(xi))

    def jl_inv(self, xi: torch.Tensor) -> torch.Tensor:
        # Jl(xi) = Jr(-xi)
        return torch.linalg.inv(right_jacobian(self.ad(-xi)))

    def retract(self, X: torch.Tensor, delta: torch.Tensor) -> torch.Tensor:
        """X * Exp(delta)  (right retraction of Appendix D)."""
        return X @ self.exp(delta)


SE2 = Group("SE2")
SE3 = Group("SE3")


def group(name: str) -> Group:
    return SE3 if name == "SE3" else SE2


__all__ = [n for n in dir() if not n.startswith("_")] + ["math"]
