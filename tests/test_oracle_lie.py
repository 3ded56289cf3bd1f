"""Pins of the oracle's Lie-group maps against library routines, finite
differences and group identities (Appendix D; right perturbations)."""
import numpy as np
import pytest
import scipy.linalg
import torch
from scipy.spatial.transform import Rotation

from oracle import lie

DT = torch.float64
rng = np.random.default_rng(1234)


def _rand_xi6(n, max_angle=np.pi - 1e-3, scale_t=3.0):
    axis = rng.normal(size=(n, 3))
    axis /= np.linalg.norm(axis, axis=1, keepdims=True)
    ang = rng.uniform(0, max_angle, size=(n, 1))
    # include tiny and near-pi angles
    ang[0] = 1e-9
    ang[1] = 3e-5
    ang[2] = max_angle
    return torch.as_tensor(np.hstack([scale_t * rng.normal(size=(n, 3)), axis * ang]), dtype=DT)


def _rand_se3(n):
    R = Rotation.random(n, random_state=7).as_matrix()
    T = np.zeros((n, 4, 4))
    T[:, :3, :3] = R
    T[:, :3, 3] = 5 * rng.normal(size=(n, 3))
    T[:, 3, 3] = 1
    return torch.as_tensor(T, dtype=DT)


def test_se3_exp_matches_expm():
    xi = _rand_xi6(64)
    ours = lie.se3_exp(xi)
    ref = np.stack([scipy.linalg.expm(lie.se3_hat(x).numpy()) for x in xi])
    assert np.abs(ours.numpy() - ref).max() < 1e-12 * max(1, np.abs(ref).max())


def test_se2_exp_matches_expm():
    xi = torch.as_tensor(np.hstack([3 * rng.normal(size=(64, 2)), rng.uniform(-np.pi, np.pi, (64, 1))]), dtype=DT)
    xi[0, 2] = 1e-10
    ours = lie.se2_exp(xi)
    ref = np.stack([scipy.linalg.expm(lie.se2_hat(x).numpy()) for x in xi])
    assert np.abs(ours.numpy() - ref).max() < 1e-12 * max(1, np.abs(ref).max())


def test_se2_embeds_in_se3():
    xi = torch.as_tensor(np.hstack([rng.normal(size=(16, 2)), rng.uniform(-3, 3, (16, 1))]), dtype=DT)
    xi6 = torch.zeros(16, 6, dtype=DT)
    xi6[:, :2] = xi[:, :2]
    xi6[:, 5] = xi[:, 2]
    T3 = lie.se3_exp(xi6)
    T2 = lie.se2_exp(xi)
    assert torch.allclose(T3[:, :2, :2], T2[:, :2, :2], atol=1e-13)
    assert torch.allclose(T3[:, :2, 3], T2[:, :2, 2], atol=1e-13)


def test_se3_log_exp_roundtrip():
    xi = _rand_xi6(256)
    back = lie.se3_log(lie.se3_exp(xi))
    err = (back - xi).abs().max(-1).values
    ang = xi[:, 3:].norm(dim=-1)
    assert float(err[ang < np.pi - 1e-2].max()) < 1e-11
    assert float(err.max()) < 1e-8


def test_se3_exp_log_roundtrip_random_elements():
    T = _rand_se3(256)
    back = lie.se3_exp(lie.se3_log(T))
    assert float((back - T).abs().max()) < 1e-11


def test_so3_log_near_pi():
    axis = rng.normal(size=(32, 3))
    axis /= np.linalg.norm(axis, axis=1, keepdims=True)
    for eps in [1e-2, 1e-5, 1e-8]:
        w = torch.as_tensor(axis * (np.pi - eps), dtype=DT)
        R = lie.so3_exp(w)
        back = lie.so3_log(R)
        assert float((lie.so3_exp(back) - R).abs().max()) < 1e-10
        assert float((back.norm(dim=-1) - (np.pi - eps)).abs().max()) < 1e-8


def test_se2_log_exp_roundtrip():
    xi = torch.as_tensor(np.hstack([3 * rng.normal(size=(128, 2)), rng.uniform(-np.pi + 1e-6, np.pi - 1e-6, (128, 1))]), dtype=DT)
    assert float((lie.se2_log(lie.se2_exp(xi)) - xi).abs().max()) < 1e-11


@pytest.mark.parametrize("G", [lie.SE2, lie.SE3])
def test_adjoint_identity(G):
    n = 32
    if G is lie.SE3:
        X = _rand_se3(n)
        xi = _rand_xi6(n, max_angle=2.0)
    else:
        X = lie.se2_exp(torch.as_tensor(rng.normal(size=(n, 3)) * 2, dtype=DT))
        xi = torch.as_tensor(rng.normal(size=(n, 3)), dtype=DT)
    lhs = X @ G.exp(xi) @ G.inv(X)
    rhs = G.exp((G.Ad(X) @ xi[..., None])[..., 0])
    assert float((lhs - rhs).abs().max()) < 1e-11


@pytest.mark.parametrize("G", [lie.SE2, lie.SE3])
def test_ad_is_bracket(G):
    a = torch.as_tensor(rng.normal(size=(16, G.dof)), dtype=DT)
    b = torch.as_tensor(rng.normal(size=(16, G.dof)), dtype=DT)
    A, Bm = G.hat(a), G.hat(b)
    lhs = G.vee(A @ Bm - Bm @ A)
    rhs = (G.ad(a) @ b[..., None])[..., 0]
    assert float((lhs - rhs).abs().max()) < 1e-13


@pytest.mark.parametrize("G", [lie.SE2, lie.SE3])
def test_right_jacobian_finite_difference(G):
    """Log(Exp(xi)^-1 Exp(xi + h e_k)) / h -> Jr(xi) e_k (central differences)."""
    n, h = 16, 1e-6
    if G is lie.SE3:
        xi = _rand_xi6(n, max_angle=2.5, scale_t=2.0)
    else:
        xi = torch.as_tensor(np.hstack([2 * rng.normal(size=(n, 2)), rng.uniform(-2.5, 2.5, (n, 1))]), dtype=DT)
    Jr = G.jr(xi)
    X0inv = G.inv(G.exp(xi))
    for k in range(G.dof):
        e = torch.zeros(G.dof, dtype=DT)
        e[k] = h
        fd = (G.log(X0inv @ G.exp(xi + e)) - G.log(X0inv @ G.exp(xi - e))) / (2 * h)
        assert float((fd - Jr[..., k]).abs().max()) < 1e-7 * max(1.0, float(Jr.abs().max()))
    I = torch.eye(G.dof, dtype=DT)
    assert float((G.jr_inv(xi) @ Jr - I).abs().max()) < 1e-12


def test_right_jacobian_so3_closed_form_block():
    """The rotation block of the SE(3) series equals the textbook SO(3) Jr."""
    xi = _rand_xi6(16, max_angle=2.5)
    Jr = lie.SE3.jr(xi)
    phi = xi[:, 3:]
    th = phi.norm(dim=-1)[:, None, None]
    W = lie.so3_hat(phi)
    ref = torch.eye(3, dtype=DT) - (1 - torch.cos(th)) / th ** 2 * W + (th - torch.sin(th)) / th ** 3 * W @ W
    assert float((Jr[:, 3:, 3:] - ref)[3:].abs().max()) < 1e-12
    assert float(Jr[:, 3:, :3].abs().max()) == 0.0
