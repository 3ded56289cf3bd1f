"""Pins of the oracle's cost functions: analytic Jacobians against central
finite differences on right perturbations, zero residual on noiseless data,
and the Huber loss against its definition."""
import numpy as np
import pytest
import torch

import synth
from oracle import costs, lie
from oracle import solve as S

DT = torch.float64
rng = np.random.default_rng(99)
H = 1e-6


def _rand_pose(G, n, scale=2.0):
    if G is lie.SE3:
        xi = np.hstack([scale * rng.normal(size=(n, 3)), rng.normal(size=(n, 3))])
    else:
        xi = np.hstack([scale * rng.normal(size=(n, 2)), rng.uniform(-3, 3, (n, 1))])
    return G.exp(torch.as_tensor(xi, dtype=DT))


def _basis(d, k):
    e = torch.zeros(d, dtype=DT)
    e[k] = H
    return e


@pytest.mark.parametrize("G", [lie.SE2, lie.SE3])
def test_between_jacobians_fd(G):
    n = 24
    Xi, Xj = _rand_pose(G, n), _rand_pose(G, n)
    # measurement close to the relative pose so that c is a residual, plus far cases
    Z = G.inv(Xi) @ Xj @ G.exp(torch.as_tensor(0.3 * rng.normal(size=(n, G.dof)), dtype=DT))
    c, Ci, Cj = costs.between(G, Xi, Xj, Z)
    for k in range(G.dof):
        e = _basis(G.dof, k)
        fdi = (costs.between(G, G.retract(Xi, e), Xj, Z)[0] - costs.between(G, G.retract(Xi, -e), Xj, Z)[0]) / (2 * H)
        fdj = (costs.between(G, Xi, G.retract(Xj, e), Z)[0] - costs.between(G, Xi, G.retract(Xj, -e), Z)[0]) / (2 * H)
        scale = max(1.0, float(Ci.abs().max()))
        assert float((fdi - Ci[..., k]).abs().max()) < 1e-7 * scale
        assert float((fdj - Cj[..., k]).abs().max()) < 1e-7 * scale


@pytest.mark.parametrize("G", [lie.SE2, lie.SE3])
def test_prior_jacobian_fd(G):
    X, P = _rand_pose(G, 16), _rand_pose(G, 16)
    c, C = costs.prior(G, X, P)
    for k in range(G.dof):
        e = _basis(G.dof, k)
        fd = (costs.prior(G, G.retract(X, e), P)[0] - costs.prior(G, G.retract(X, -e), P)[0]) / (2 * H)
        assert float((fd - C[..., k]).abs().max()) < 1e-7 * max(1.0, float(C.abs().max()))


def test_reprojection_jacobians_fd():
    n = 32
    T = lie.se3_exp(torch.as_tensor(np.hstack([0.3 * rng.normal(size=(n, 3)), 0.2 * rng.normal(size=(n, 3))]), dtype=DT))
    p = torch.as_tensor(rng.normal(size=(n, 3)) + np.array([0, 0, 6.0]), dtype=DT)
    uv = torch.as_tensor(rng.uniform(0, 600, size=(n, 2)), dtype=DT)
    intr = (500.0, 480.0, 320.0, 240.0)
    c, Cc, Cp = costs.reprojection(T, p, uv, intr)
    for k in range(6):
        e = _basis(6, k)
        fd = (costs.reprojection(lie.SE3.retract(T, e), p, uv, intr)[0] -
              costs.reprojection(lie.SE3.retract(T, -e), p, uv, intr)[0]) / (2 * H)
        assert float((fd - Cc[..., k]).abs().max()) < 1e-7 * float(Cc.abs().max())
    for k in range(3):
        e = _basis(3, k)
        fd = (costs.reprojection(T, p + e, uv, intr)[0] - costs.reprojection(T, p - e, uv, intr)[0]) / (2 * H)
        assert float((fd - Cp[..., k]).abs().max()) < 1e-7 * float(Cp.abs().max())


def test_huber_definition():
    d = 2.0
    s = torch.tensor([0.0, 1.0, 3.9, 4.0, 4.1, 100.0], dtype=DT)
    rho, drho = costs.huber(s, d)
    ref = torch.where(s <= 4.0, s, 2 * d * torch.sqrt(s) - 4.0)
    assert torch.allclose(rho, ref, atol=0, rtol=0)
    # continuity of rho and rho' at s = delta^2
    lo, hi = costs.huber(torch.tensor([4.0 - 1e-9, 4.0 + 1e-9], dtype=DT), d)
    assert abs(float(lo[1] - lo[0])) < 1e-8 and abs(float(hi[1] - hi[0])) < 1e-8
    # rho' = d rho / ds away from the kink
    for s0 in [1.0, 9.0, 50.0]:
        fd = (costs.huber(torch.tensor(s0 + H, dtype=DT), d)[0] - costs.huber(torch.tensor(s0 - H, dtype=DT), d)[0]) / (2 * H)
        assert abs(float(fd - costs.huber(torch.tensor(s0, dtype=DT), d)[1])) < 1e-8


@pytest.mark.parametrize("make", [
    lambda: synth.circle_se2(noiseless=True),
    lambda: synth.walk_se3(batch=2, n_poses=12, n_loops=6, noiseless=True),
])
def test_noiseless_graph_zero_residual_and_step(make):
    p = make()
    for b, g in enumerate(S.graphs_of(p, poses=p["poses_gt"])):
        lin = S.linearize_pose_graph(g, g.X)
        assert float(lin.S) < 1e-24
        assert float(lin.g.abs().max()) < 1e-12
        delta, _ = S.pose_graph_step(lin, 0.0)
        assert float(delta.abs().max()) < 1e-12


def test_noiseless_ba_zero_residual_and_step():
    p = synth.bundle_adjustment(batch=1, n_cams=8, n_points=48, obs_per_point=4, radius=10.0,
                                noiseless=True)
    g = S.graphs_of(p, poses=p["poses_gt"], points=p["points_gt"])[0]
    lin = S.linearize_ba(g, g.X, g.pts)
    assert float(lin.S) < 1e-20
    L, Ci, EC = S.schur_factor(lin, 0.0)
    dc, dp = S.schur_solve(lin, L, Ci, EC, lin.g, lin.gp)
    assert float(dc.abs().max()) < 1e-10 and float(dp.abs().max()) < 1e-10
