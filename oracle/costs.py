"""Cost functions of the oracle: residuals and their Jacobians.

A residual is r_i = w_i c_i (Eq. nls) with a scalar weight w_i = exp(l_i)
(the paper's ScaleCostWeight, parameterised by its logarithm so that it stays
positive).  Jacobians C_i = dc_i/dtheta are taken with respect to right
perturbations X*Exp(delta) (Appendix D, Eq. grad1), in the tangent order of
``oracle.lie``.

* relative pose ("coordinate-independent relative pose error", Appendix E.1):
  c = Log(Z^-1 X_i^-1 X_j)
  dc/d(delta_j) = Jr^-1(c)
  dc/d(delta_i) = -Jr^-1(c) Ad(X_j^-1 X_i)
* prior (Gaussian measurement of one pose): c = Log(P^-1 X), dc/d(delta) = Jr^-1(c)
* pinhole reprojection (Appendix E.3) of world point p by world-to-camera
  pose T: p_c = R p + t, c = (fx x/z + cx, fy y/z + cy) - uv,
  dc/d(delta_T) = dpi/dp_c R [I, -p^],  dc/dp = dpi/dp_c R
* Huber robust loss on s = ||r||^2 (used by the bundle-adjustment workload):
  rho(s) = s for s <= d^2, 2 d sqrt(s) - d^2 otherwise; the step uses the
  first-order reweighting rho'(s) (no rho'' term).
"""
from __future__ import annotations

import torch

from . import lie

DT = torch.float64


def between(G: lie.Group, Xi: torch.Tensor, Xj: torch.Tensor, Z: torch.Tensor):
    """Relative-pose cost; returns (c, C_i, C_j)."""
    E = G.inv(Z) @ G.inv(Xi) @ Xj
    c = G.log(E)
    Jri = G.jr_inv(c)
    Cj = Jri
    Ci = -Jri @ G.Ad(G.inv(Xj) @ Xi)
    return c, Ci, Cj


def prior(G: lie.Group, X: torch.Tensor, P: torch.Tensor):
    """Prior (Gaussian measurement) on one pose; returns (c, C)."""
    c = G.log(G.inv(P) @ X)
    return c, G.jr_inv(c)


def reprojection(T: torch.Tensor, p: torch.Tensor, uv: torch.Tensor, intr):
    """Pinhole reprojection of world point p by world-to-camera T; returns
    (c [...,2], C_cam [...,2,6], C_pt [...,2,3])."""
    fx, fy, cx, cy = intr
    R = T[..., :3, :3]
    pc = (R @ p[..., None])[..., 0] + T[..., :3, 3]
    x, y, z = pc[..., 0], pc[..., 1], pc[..., 2]
    u = fx * x / z + cx
    v = fy * y / z + cy
    c = torch.stack([u, v], -1) - uv
    zero = torch.zeros_like(z)
    dpi = torch.stack([torch.stack([fx / z, zero, -fx * x / (z * z)], -1),
                       torch.stack([zero, fy / z, -fy * y / (z * z)], -1)], -2)
    dR = dpi @ R
    I = torch.eye(3, dtype=DT).expand(R.shape)
    Ccam = dR @ torch.cat([I, -lie.so3_hat(p)], -1)
    return c, Ccam, dR


def huber(s: torch.Tensor, delta: float):
    """rho(s) and rho'(s) on the squared norm s (inside branch for s <= delta^2)."""
    inside = s <= delta * delta
    s_safe = torch.where(inside, torch.ones_like(s), s)
    rho = torch.where(inside, s, 2 * delta * torch.sqrt(s_safe) - delta * delta)
    drho = torch.where(inside, torch.ones_like(s), delta / torch.sqrt(s_safe))
    return rho, drho
