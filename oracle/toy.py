"""Euclidean problems with closed-form answers, run through the oracle's
normal-equation / Cholesky step (``solve.pose_graph_step``) and the same
Proposition-1 recipe as ``solve.implicit_grad_graph``.

* curve fit of Listing 1 / Appendix B: residuals r_i = y_i - v exp(x_i) with
  one scalar variable v and auxiliary data (x, y); the problem is linear in
  v, so one Gauss-Newton step from any v0 lands on v* = sum y e^x / sum e^2x.
* linear-Gaussian least squares r = W (A theta - b): one Gauss-Newton step
  lands on the weighted least-squares solution.
"""
from __future__ import annotations

import torch

from .solve import Lin, pose_graph_step

DT = torch.float64


def gauss_newton(residual, theta0: torch.Tensor, iterations: int, lam: float = 0.0):
    """Generic GN/LM on a Euclidean vector: J from autograd, H = J^T J, g = J^T r,
    theta <- theta - (H + lam I)^-1 g."""
    theta = theta0.clone()
    for _ in range(iterations):
        r = residual(theta)
        J = torch.autograd.functional.jacobian(residual, theta)
        lin = Lin(S=0.5 * (r * r).sum(), H=J.T @ J, g=J.T @ r)
        delta, _ = pose_graph_step(lin, lam)
        theta = theta - delta
    return theta


def implicit_grad(residual_of, theta_star: torch.Tensor, phi: torch.Tensor, v: torch.Tensor):
    """dL/dphi = -d/dphi [u^T g(theta*; phi)], u = H^-1 v with H = J^T J at theta*
    (Proposition 1 with the Gauss-Newton Hessian in the stopped slot)."""
    r_fn = lambda th: residual_of(th, phi)
    J = torch.autograd.functional.jacobian(r_fn, theta_star)
    H = J.T @ J
    u = torch.linalg.solve(H, v)
    p = phi.clone().requires_grad_(True)
    th = theta_star.clone().requires_grad_(True)
    r = residual_of(th, p)
    # g(theta; phi) = J^T r = d/dtheta (1/2 |r|^2), kept differentiable in phi
    (g,) = torch.autograd.grad(0.5 * (r * r).sum(), [th], create_graph=True)
    (dphi,) = torch.autograd.grad((g * u).sum(), [p])
    return -dphi


def curve_fit_residual(v: torch.Tensor, x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    return y - v[0] * torch.exp(x)


def linear_gaussian_residual(theta, A, b, w):
    return w * (A @ theta - b)
