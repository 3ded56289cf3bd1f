"""Pins of the oracle's bundle-adjustment normal equations (linearize_ba)
against quantities obtained without its analytic blocks.

The reprojection residual is re-derived here from the pinhole model of the
paper's BA example (App. E.3), the camera perturbation is the right
perturbation T Exp(xi) of App. D written with the library matrix exponential
of the 4x4 twist, and every Jacobian, gradient and Hessian comes from
torch.autograd.  So a dropped robust weight, a wrong sign or a transposed
block in linearize_ba (camera block B, camera-point block E, point blocks C,
gradients g_c, g_p) fails one of these tests.

* With both Huber branches active, B, E, C equal sum_o rho'(s_o) J_o^T J_o
  (plus the prior terms) built from autograd Jacobians of the residuals
  w_o c_o, and (g_c, g_p) equals the autograd gradient of
  S = 1/2 sum rho(s) (Eq. nls with the robust loss; the gradient is exact,
  the matrix is the first-order reweighted Gauss-Newton one).
* On a noiseless problem (zero residual, all observations in the quadratic
  branch) the full camera + point matrix equals the autograd Hessian of S:
  there the Gauss-Newton matrix is the exact Hessian.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import lie
from oracle import solve as S

DT = torch.float64


def _twist_hat(xi):
    """4x4 matrix of a twist [rho; phi] (translation first)."""
    rho, phi = xi[..., :3], xi[..., 3:]
    z = torch.zeros_like(phi[..., 0])
    W = torch.stack([torch.stack([z, -phi[..., 2], phi[..., 1]], -1),
                     torch.stack([phi[..., 2], z, -phi[..., 0]], -1),
                     torch.stack([-phi[..., 1], phi[..., 0], z], -1)], -2)
    top = torch.cat([W, rho[..., :, None]], -1)
    bottom = torch.zeros(*xi.shape[:-1], 1, 4, dtype=xi.dtype)
    return torch.cat([top, bottom], -2)


def _residuals(g, x, w_o=None, prior_at_identity=False):
    """Per-observation weighted reprojection residuals [O, 2] and prior
    residuals [P, 6] at the perturbation x = [xi_cam (6 Nc); dp (3 Np)].
    With prior_at_identity (the prior measurement equals the camera, so the
    prior residual Log(P^-1 T Exp(xi)) is Log(Exp(xi)) = xi) the prior
    residual is xi itself, which keeps the second derivatives of the
    logarithm's angle at the identity out of the autograd Hessian."""
    Nc, Np = g.X.shape[0], g.pts.shape[0]
    xi = x[:6 * Nc].reshape(Nc, 6)
    dp = x[6 * Nc:].reshape(Np, 3)
    T = g.X @ torch.linalg.matrix_exp(_twist_hat(xi))
    P = g.pts + dp
    fx, fy, cx, cy = g.intr
    Tc = T[g.oc]
    pc = (Tc[:, :3, :3] @ P[g.op][:, :, None])[:, :, 0] + Tc[:, :3, 3]
    uv = torch.stack([fx * pc[:, 0] / pc[:, 2] + cx, fy * pc[:, 1] / pc[:, 2] + cy], -1)
    w = g.w_o if w_o is None else w_o
    r_obs = w[:, None] * (uv - g.uv)
    if prior_at_identity:
        r_pri = torch.exp(g.logw_p)[:, None] * xi[g.pv]
    else:
        r_pri = torch.exp(g.logw_p)[:, None] * lie.SE3.log(lie.SE3.inv(g.PZ) @ T[g.pv])
    return r_obs, r_pri


def _huber_rho(s, delta):
    """Huber on the squared norm, written from its definition (the square
    root only sees the outside branch, so its derivative stays finite at 0)."""
    inside = s <= delta * delta
    root = torch.sqrt(torch.where(inside, torch.ones_like(s), s))
    return torch.where(inside, s, 2.0 * delta * root - delta * delta)


def _objective(g, x, prior_at_identity=False):
    r_obs, r_pri = _residuals(g, x, prior_at_identity=prior_at_identity)
    return 0.5 * _huber_rho((r_obs ** 2).sum(-1), g.delta).sum() + 0.5 * (r_pri ** 2).sum()


def _full(lin):
    return S.ba_full_system(lin)


def _setup(noiseless, seed=3):
    p = synth.bundle_adjustment(batch=1, n_cams=6, n_points=24, obs_per_point=4, noiseless=noiseless,
                                cam_r=0.0 if noiseless else 0.002, cam_t=0.0 if noiseless else 0.005,
                                pixel_sigma=0.0 if noiseless else 2.0, seed=seed)
    g = S.graphs_of(p)[0]
    g.w_o = torch.as_tensor(np.random.default_rng(seed).uniform(0.6, 1.4, size=len(g.oc)), dtype=DT)
    return g


def test_linearize_ba_blocks_are_robust_gauss_newton_of_autograd_jacobians():
    g = _setup(noiseless=False)
    Nc, Np = g.X.shape[0], g.pts.shape[0]
    n = 6 * Nc + 3 * Np
    x0 = torch.zeros(n, dtype=DT)
    r_obs, r_pri = _residuals(g, x0)
    s = (r_obs ** 2).sum(-1)
    inside = s <= g.delta ** 2
    # both branches of the robust loss are exercised
    assert int(inside.sum()) >= 5 and int((~inside).sum()) >= 5, (int(inside.sum()), int((~inside).sum()))
    J_obs = torch.autograd.functional.jacobian(lambda x: _residuals(g, x)[0], x0)     # [O, 2, n]
    J_pri = torch.autograd.functional.jacobian(lambda x: _residuals(g, x)[1], x0)     # [P, 6, n]
    # rho'(s) by autograd of the robust loss at each observation's s
    s_req = s.clone().requires_grad_(True)
    (drho,) = torch.autograd.grad(_huber_rho(s_req, g.delta).sum(), [s_req])
    H_ref = torch.einsum("o,oan,oam->nm", drho, J_obs, J_obs) + torch.einsum("pan,pam->nm", J_pri, J_pri)
    x_req = x0.clone().requires_grad_(True)
    (g_ref,) = torch.autograd.grad(_objective(g, x_req), [x_req])

    lin = S.linearize_ba(g, g.X, g.pts)
    Hf = _full(lin)
    gf = torch.cat([lin.g, lin.gp.reshape(-1)])
    scale = float(H_ref.abs().max())
    assert float((Hf - H_ref).abs().max()) < 1e-9 * scale
    assert float((gf - g_ref).abs().max()) < 1e-9 * float(g_ref.abs().max())
    # each block separately, with the reference's own block boundaries
    nc = 6 * Nc
    assert float((lin.H - H_ref[:nc, :nc]).abs().max()) < 1e-9 * scale
    assert float((lin.E - H_ref[:nc, nc:]).abs().max()) < 1e-9 * scale
    for k in range(Np):
        blk = H_ref[nc + 3 * k: nc + 3 * k + 3, nc + 3 * k: nc + 3 * k + 3]
        assert float((lin.C[k] - blk).abs().max()) < 1e-9 * scale
    # the objective value is the robust one
    assert abs(float(lin.S) - float(_objective(g, x0))) < 1e-12 * float(lin.S)


def test_linearize_ba_equals_autograd_hessian_at_zero_residual():
    g = _setup(noiseless=True)
    Nc, Np = g.X.shape[0], g.pts.shape[0]
    n = 6 * Nc + 3 * Np
    x0 = torch.zeros(n, dtype=DT)
    r_obs, r_pri = _residuals(g, x0)
    assert float(r_obs.abs().max()) < 1e-9 and float(r_pri.abs().max()) < 1e-9
    assert float((lie.SE3.inv(g.PZ) @ g.X[g.pv] - torch.eye(4, dtype=DT)).abs().max()) < 1e-12
    H_exact = torch.autograd.functional.hessian(lambda x: _objective(g, x, prior_at_identity=True), x0)
    lin = S.linearize_ba(g, g.X, g.pts)
    Hf = _full(lin)
    scale = float(H_exact.abs().max())
    assert float((Hf - H_exact).abs().max()) < 1e-8 * scale
    assert float(torch.cat([lin.g, lin.gp.reshape(-1)]).abs().max()) < 1e-8


def test_ba_schur_step_solves_the_autograd_system():
    """The Schur elimination's step solves (H + lambda I) delta = g with H and g
    from the autograd construction above, so the point back-substitution and
    the camera system are pinned independently of linearize_ba's blocks."""
    g = _setup(noiseless=False, seed=8)
    Nc, Np = g.X.shape[0], g.pts.shape[0]
    n = 6 * Nc + 3 * Np
    x0 = torch.zeros(n, dtype=DT)
    r_obs, _ = _residuals(g, x0)
    s = (r_obs ** 2).sum(-1)
    J_obs = torch.autograd.functional.jacobian(lambda x: _residuals(g, x)[0], x0)
    J_pri = torch.autograd.functional.jacobian(lambda x: _residuals(g, x)[1], x0)
    s_req = s.clone().requires_grad_(True)
    (drho,) = torch.autograd.grad(_huber_rho(s_req, g.delta).sum(), [s_req])
    H_ref = torch.einsum("o,oan,oam->nm", drho, J_obs, J_obs) + torch.einsum("pan,pam->nm", J_pri, J_pri)
    x_req = x0.clone().requires_grad_(True)
    (g_ref,) = torch.autograd.grad(_objective(g, x_req), [x_req])
    lam = 1e-3
    want = torch.linalg.solve(H_ref + lam * torch.eye(n, dtype=DT), g_ref)
    lin = S.linearize_ba(g, g.X, g.pts)
    L, Ci, EC = S.schur_factor(lin, lam)
    dc, dp = S.schur_solve(lin, L, Ci, EC, lin.g, lin.gp)
    got = torch.cat([dc, dp.reshape(-1)])
    assert float((got - want).abs().max()) < 1e-8 * float(want.abs().max())
