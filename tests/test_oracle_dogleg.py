"""Pins of the oracle's dogleg step (oracle.solve.dogleg_step) by properties
that follow from the definition of Powell's dogleg (a trust-region method
among the paper's optimizers, Section 3), not by restating its formulas.

For the quadratic model m(d) = S - g^T d + 1/2 d^T A d with A = H + lambda I
symmetric positive definite, the Gauss-Newton point d_gn = A^-1 g, and the
Cauchy point d_c (the minimiser of m along g), the dogleg path runs from 0
to d_c and on to d_gn.  The step for a radius r is:
  * d_gn when ||d_gn|| <= r;
  * the gradient direction cut at the boundary when ||d_c|| >= r;
  * otherwise the point of the segment [d_c, d_gn] at distance r.
Checked here on random SPD systems: the radius is met exactly, the segment
point lies on the segment (d = d_c + beta (d_gn - d_c), beta in [0, 1]),
the Cauchy point is the minimiser along g (found by a scalar minimisation,
not by its closed form), the model decrease is at least the Cauchy point's
(or the cut gradient's), is non-increasing in m along the path as r grows,
and the step is continuous where the branches meet.
"""
import numpy as np
import pytest
import torch
from scipy.optimize import minimize_scalar

from oracle import solve as S

DT = torch.float64


def _system(n, seed, cond=1e3):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    ev = np.logspace(0, np.log10(cond), n)
    H = (Q * ev) @ Q.T
    g = rng.normal(size=n)
    return H, g


def _lin(H, g):
    return S.Lin(S=torch.tensor(10.0, dtype=DT), H=torch.as_tensor(H, dtype=DT), g=torch.as_tensor(g, dtype=DT))


def _model_decrease(A, g, d):
    return g @ d - 0.5 * d @ A @ d


def _cauchy_point(A, g):
    """Minimiser of the model along +g, by a bounded scalar search."""
    f = lambda t: -_model_decrease(A, g, t * g)
    hi = 10.0 / np.linalg.norm(g) * np.linalg.norm(np.linalg.solve(A, g))
    res = minimize_scalar(f, bounds=(0.0, hi), method="bounded", options=dict(xatol=1e-14))
    return res.x * g


@pytest.mark.parametrize("seed,n,lam", [(0, 6, 0.0), (1, 12, 1e-3), (2, 30, 0.5)])
def test_dogleg_segment_branch_properties(seed, n, lam):
    H, g = _system(n, seed)
    A = H + lam * np.eye(n)
    d_gn = np.linalg.solve(A, g)
    d_c = _cauchy_point(A, g)
    nc, ngn = np.linalg.norm(d_c), np.linalg.norm(d_gn)
    assert nc < ngn                              # a non-empty segment branch exists
    lin = _lin(H, g)
    prev_m = None
    for frac in (0.05, 0.3, 0.6, 0.95):
        r = nc + frac * (ngn - nc)
        d, boundary, pred = S.dogleg_step(lin, None, torch.as_tensor(d_gn, dtype=DT), lam, r)
        d = d.numpy()
        assert boundary
        assert abs(np.linalg.norm(d) - r) < 1e-12 * r
        # on the segment from the Cauchy point to the Gauss-Newton point
        seg = d_gn - d_c
        beta = (d - d_c) @ seg / (seg @ seg)
        assert -1e-9 <= beta <= 1.0 + 1e-9
        assert np.linalg.norm(d - (d_c + beta * seg)) < 1e-7 * np.linalg.norm(d)
        # predicted decrease: the model's, and at least the Cauchy point's
        m = _model_decrease(A, g, d)
        assert abs(pred - m) < 1e-12 * abs(m)
        assert m >= _model_decrease(A, g, d_c) * (1 - 1e-12)
        if prev_m is not None:
            assert m >= prev_m * (1 - 1e-12)     # the model decreases along the path
        prev_m = m


@pytest.mark.parametrize("seed", [3, 4])
def test_dogleg_gradient_and_gauss_newton_branches(seed):
    n, lam = 10, 1e-2
    H, g = _system(n, seed, cond=1e4)
    A = H + lam * np.eye(n)
    d_gn = np.linalg.solve(A, g)
    d_c = _cauchy_point(A, g)
    lin = _lin(H, g)
    # radius inside the Cauchy point: the gradient cut at the boundary, which
    # beats every other point of the boundary along g
    r = 0.5 * np.linalg.norm(d_c)
    d, boundary, pred = S.dogleg_step(lin, None, torch.as_tensor(d_gn, dtype=DT), lam, r)
    d = d.numpy()
    assert boundary
    assert abs(np.linalg.norm(d) - r) < 1e-12 * r
    assert np.linalg.norm(d / r - g / np.linalg.norm(g)) < 1e-12
    assert _model_decrease(A, g, d) > 0
    # radius beyond the Gauss-Newton point: the Gauss-Newton step, not on the boundary
    d, boundary, pred = S.dogleg_step(lin, None, torch.as_tensor(d_gn, dtype=DT), lam,
                                      1.5 * np.linalg.norm(d_gn))
    assert not boundary
    assert np.abs(d.numpy() - d_gn).max() < 1e-14 * np.abs(d_gn).max()
    assert abs(pred - 0.5 * g @ d_gn) < 1e-10 * abs(pred)   # the minimum of the model


def test_dogleg_is_continuous_where_branches_meet():
    n, lam = 8, 0.0
    H, g = _system(n, 5)
    d_gn = np.linalg.solve(H, g)
    d_c = _cauchy_point(H, g)
    lin = _lin(H, g)
    gn = torch.as_tensor(d_gn, dtype=DT)
    nc, ngn = np.linalg.norm(d_c), np.linalg.norm(d_gn)
    for r, want in ((nc, d_c), (ngn, d_gn)):
        lo = S.dogleg_step(lin, None, gn, lam, r * (1 - 1e-9))[0].numpy()
        hi = S.dogleg_step(lin, None, gn, lam, r * (1 + 1e-9))[0].numpy()
        assert np.linalg.norm(lo - want) < 1e-6 * np.linalg.norm(want)
        assert np.linalg.norm(hi - want) < 1e-6 * np.linalg.norm(want)
