"""Pins of the oracle's inner loop and implicit backward:
closed-form Euclidean problems, the LM step against a direct solve, the Schur
step against the full system, and Proposition 1 against finite differences of
the stopped Newton step and of the fully re-solved problem."""
import numpy as np
import pytest
import torch

import synth
from oracle import lie, toy
from oracle import solve as S

DT = torch.float64
rng = np.random.default_rng(2024)


# ---------------------------------------------------------------------------
# Euclidean problems with closed forms
# ---------------------------------------------------------------------------
def test_linear_gaussian_one_step_is_least_squares():
    A = torch.as_tensor(rng.normal(size=(40, 7)), dtype=DT)
    b = torch.as_tensor(rng.normal(size=40), dtype=DT)
    w = torch.as_tensor(rng.uniform(0.5, 2.0, size=40), dtype=DT)
    theta0 = torch.as_tensor(rng.normal(size=7), dtype=DT)
    one = toy.gauss_newton(lambda th: toy.linear_gaussian_residual(th, A, b, w), theta0, 1)
    ref = np.linalg.lstsq((w[:, None] * A).numpy(), (w * b).numpy(), rcond=None)[0]
    assert np.abs(one.numpy() - ref).max() < 1e-12


def test_linear_gaussian_weight_gradient_closed_form():
    """theta*(w) = (A^T W^2 A)^-1 A^T W^2 b; its derivative against Prop. 1
    (the Gauss-Newton Hessian is the exact Hessian for a linear problem)."""
    A = torch.as_tensor(rng.normal(size=(12, 3)), dtype=DT)
    b = torch.as_tensor(rng.normal(size=12), dtype=DT)
    w = torch.as_tensor(rng.uniform(0.5, 2.0, size=12), dtype=DT)
    v = torch.as_tensor(rng.normal(size=3), dtype=DT)

    def theta_star(ww):
        W2 = torch.diag(ww * ww)
        return torch.linalg.solve(A.T @ W2 @ A, A.T @ W2 @ b)

    th = theta_star(w)
    ours = toy.implicit_grad(lambda t, ww: toy.linear_gaussian_residual(t, A, b, ww), th, w, v)
    ref = torch.autograd.functional.vjp(theta_star, w, v)[1]
    assert float((ours - ref).abs().max()) < 1e-10 * max(1.0, float(ref.abs().max()))


def test_curve_fit_listing1_closed_forms():
    """Listing 1: r_i = y_i - v exp(x_i); v* = sum y e^x / sum e^2x after one
    step, and dv*/dx_k = (y_k e^x_k S2 - 2 e^2x_k S1) / S2^2 with S1 = sum y e^x,
    S2 = sum e^2x."""
    x = torch.as_tensor(rng.normal(size=20), dtype=DT)
    y = 2.0 * torch.exp(x) + torch.as_tensor(0.1 * rng.normal(size=20), dtype=DT)
    v = toy.gauss_newton(lambda vv: toy.curve_fit_residual(vv, x, y), torch.ones(1, dtype=DT), 1)
    ex, e2x = torch.exp(x), torch.exp(2 * x)
    S1, S2 = (y * ex).sum(), e2x.sum()
    assert abs(float(v[0] - S1 / S2)) < 1e-12
    # L = (v* - v_true)^2, dL/dv = 2 (v* - 2)
    dLdv = 2 * (v - 2.0)
    grad = toy.implicit_grad(lambda vv, xx: toy.curve_fit_residual(vv, xx, y), v, x, dLdv)
    ref = dLdv[0] * (y * ex * S2 - 2 * e2x * S1) / S2 ** 2
    assert float((grad - ref).abs().max()) < 1e-10 * float(ref.abs().max())


# ---------------------------------------------------------------------------
# damping and the Schur complement
# ---------------------------------------------------------------------------
def test_lm_step_equals_direct_solve_and_gn_limit():
    p = synth.walk_se3(batch=1, n_poses=10, n_loops=5)
    g = S.graphs_of(p)[0]
    lin = S.linearize_pose_graph(g, g.X)
    for lam in [1e-3, 1.0]:
        delta, _ = S.pose_graph_step(lin, lam)
        ref = np.linalg.solve(lin.H.numpy() + lam * np.eye(lin.H.shape[0]), lin.g.numpy())
        assert np.abs(delta.numpy() - ref).max() < 1e-10 * np.abs(ref).max()
    d0, _ = S.pose_graph_step(lin, 0.0)
    d1, _ = S.pose_graph_step(lin, 1e-13)
    assert float((d0 - d1).abs().max()) < 1e-6 * float(d0.abs().max())


def _small_ba(noiseless=False):
    return synth.bundle_adjustment(batch=1, n_cams=8, n_points=40, obs_per_point=4, noiseless=noiseless)


def test_adaptive_lm_ba_follows_full_system_steps():
    """Adaptive damping on bundle adjustment from a very poor start, replayed
    independently: each trial step is the damped full (cameras + points)
    system solved by numpy, the step is kept iff the objective strictly
    decreases.  The oracle's Schur path gives the same iterates, objectives
    and lambdas, and the run rejects six steps in a row and then recovers."""
    p = synth.bundle_adjustment(batch=1, n_cams=8, n_points=40, obs_per_point=4, cam_r=1.0, cam_t=3.0,
                                point_sigma=2.0, seed=2)
    g = S.graphs_of(p)[0]
    K, lam = 10, 1e-7
    r = S.solve_graph(g, K, lam, adaptive=True)
    X, pts, lams, objs = g.X.clone(), g.pts.clone(), [], []
    for _ in range(K):
        lin = S.linearize_ba(g, X, pts)
        objs.append(float(lin.S))
        lams.append(lam)
        nc, npnt = lin.H.shape[0], lin.C.shape[0]
        Hf = np.zeros((nc + 3 * npnt, nc + 3 * npnt))
        Hf[:nc, :nc] = lin.H.numpy()
        Hf[:nc, nc:] = lin.E.numpy()
        Hf[nc:, :nc] = lin.E.numpy().T
        for k in range(npnt):
            Hf[nc + 3 * k: nc + 3 * k + 3, nc + 3 * k: nc + 3 * k + 3] = lin.C[k].numpy()
        step = np.linalg.solve(Hf + lam * np.eye(Hf.shape[0]),
                               np.concatenate([lin.g.numpy(), lin.gp.numpy().reshape(-1)]))
        Xt = lie.SE3.retract(X, -torch.as_tensor(step[:nc]).reshape(-1, 6))
        pt_t = pts - torch.as_tensor(step[nc:]).reshape(-1, 3)
        if float(S.linearize_ba(g, Xt, pt_t).S) < float(lin.S):
            X, pts, lam = Xt, pt_t, max(lam / 10.0, 1e-7)
        else:
            lam = min(lam * 10.0, 1e7)
    objs.append(float(S.linearize_ba(g, X, pts).S))
    assert r.lambdas == pytest.approx(lams, rel=1e-15)
    assert np.allclose(r.objective, objs, rtol=1e-10, atol=0)
    assert (lie.SE3.to_storage(r.X) - lie.SE3.to_storage(X)).abs().max() < 1e-9
    assert (r.pts - pts).abs().max() < 1e-9
    rejected = [objs[t + 1] == objs[t] for t in range(K)]
    assert rejected[3:9] == [True] * 6 and not any(rejected[:3]) and not rejected[9]


def test_dogleg_ba_huge_radius_is_gauss_newton_and_replay():
    """Bundle-adjustment dogleg: with a huge radius every Gauss-Newton step
    is inside and kept, so it reproduces the plain solve; from a very poor
    start with radius 10, an independent replay (numpy solves of the full
    camera + point system for the Gauss-Newton point and the model) gives the
    same objectives and radii, a refused step included."""
    p = synth.bundle_adjustment(batch=1, n_cams=8, n_points=40, obs_per_point=4, seed=5)
    g = S.graphs_of(p)[0]
    a, b = S.solve_graph(g, 5, 0.0), S.solve_graph(g, 5, 0.0, dogleg_radius=1e9)
    assert a.objective == b.objective
    q = synth.bundle_adjustment(batch=1, n_cams=8, n_points=40, obs_per_point=4, cam_r=1.0, cam_t=3.0,
                                point_sigma=2.0, seed=2)
    g = S.graphs_of(q)[0]
    K, radius = 8, 10.0
    r = S.solve_graph(g, K, 0.0, dogleg_radius=radius)
    X, pts, objs, radii = g.X.clone(), g.pts.clone(), [], []
    for _ in range(K):
        lin = S.linearize_ba(g, X, pts)
        objs.append(float(lin.S))
        radii.append(radius)
        Hf = S.ba_full_system(lin).numpy()
        gv = np.concatenate([lin.g.numpy(), lin.gp.numpy().reshape(-1)])
        dgn = np.linalg.solve(Hf, gv)
        if np.linalg.norm(dgn) <= radius:
            d, on_b = dgn, False
        else:
            on_b = True
            alpha = gv @ gv / (gv @ Hf @ gv)
            if alpha * np.linalg.norm(gv) >= radius:
                d = radius / np.linalg.norm(gv) * gv
            else:
                sd, dd = alpha * gv, dgn - alpha * gv
                qa, qb, qc = dd @ dd, 2 * sd @ dd, sd @ sd - radius ** 2
                d = sd + (-qb + np.sqrt(qb * qb - 4 * qa * qc)) / (2 * qa) * dd
        pred = gv @ d - 0.5 * d @ Hf @ d
        nc = lin.H.shape[0]
        Xt = lie.SE3.retract(X, -torch.as_tensor(d[:nc]).reshape(-1, 6))
        pt_t = pts - torch.as_tensor(d[nc:]).reshape(-1, 3)
        s_trial = float(S.linearize_ba(g, Xt, pt_t).S)
        rho = (float(lin.S) - s_trial) / pred
        if s_trial < float(lin.S):
            X, pts = Xt, pt_t
        if not rho >= 0.25:
            radius = 0.25 * np.linalg.norm(d)
        elif rho > 0.75 and on_b:
            radius = min(2 * radius, 1e4)
    objs.append(float(S.linearize_ba(g, X, pts).S))
    assert np.allclose(r.objective, objs, rtol=1e-9, atol=0)
    assert np.allclose(r.radii, radii, rtol=1e-9, atol=0)
    assert any(objs[t + 1] == objs[t] for t in range(K))


@pytest.mark.parametrize("lam", [0.0, 1e-3])
def test_schur_step_equals_full_system(lam):
    p = _small_ba()
    g = S.graphs_of(p)[0]
    lin = S.linearize_ba(g, g.X, g.pts)
    L, Ci, EC = S.schur_factor(lin, lam)
    dc, dp = S.schur_solve(lin, L, Ci, EC, lin.g, lin.gp)
    nc, npnt = lin.H.shape[0], lin.C.shape[0]
    Hf = np.zeros((nc + 3 * npnt, nc + 3 * npnt))
    Hf[:nc, :nc] = lin.H.numpy()
    Hf[:nc, nc:] = lin.E.numpy()
    Hf[nc:, :nc] = lin.E.numpy().T
    for k in range(npnt):
        Hf[nc + 3 * k: nc + 3 * k + 3, nc + 3 * k: nc + 3 * k + 3] = lin.C[k].numpy()
    Hf += lam * np.eye(Hf.shape[0])
    ref = np.linalg.solve(Hf, np.concatenate([lin.g.numpy(), lin.gp.numpy().reshape(-1)]))
    got = np.concatenate([dc.numpy(), dp.numpy().reshape(-1)])
    assert np.abs(got - ref).max() < 1e-9 * np.abs(ref).max()


# ---------------------------------------------------------------------------
# Proposition 1 against finite differences of the stopped Newton step:
# F(phi) = v^T (-Hbar^-1 g(theta_K; phi)) with Hbar frozen has dF/dphi equal
# to the implicit gradient exactly.
# ---------------------------------------------------------------------------
def _fd_stopped_newton(g, res, v, which, h=1e-6):
    (L,) = res.factor
    d = g.G.dof

    def F(le, lp, tau):
        lin = S.linearize_pose_graph(g, res.X, tau=tau, logw_e=le, logw_p=lp)
        return float(-(v.reshape(-1) * torch.cholesky_solve(lin.g[:, None], L)[:, 0]).sum())

    le0, lp0 = g.logw_e.clone(), g.logw_p.clone()
    tau0 = torch.zeros(len(g.ei), d, dtype=DT)
    out = []
    if which == "edge_logw":
        for k in range(len(le0)):
            a, b_ = le0.clone(), le0.clone()
            a[k] += h
            b_[k] -= h
            out.append((F(a, lp0, tau0) - F(b_, lp0, tau0)) / (2 * h))
    elif which == "prior_logw":
        for k in range(len(lp0)):
            a, b_ = lp0.clone(), lp0.clone()
            a[k] += h
            b_[k] -= h
            out.append((F(le0, a, tau0) - F(le0, b_, tau0)) / (2 * h))
    else:
        for k in range(len(le0)):
            row = []
            for j in range(d):
                a, b_ = tau0.clone(), tau0.clone()
                a[k, j] += h
                b_[k, j] -= h
                row.append((F(le0, lp0, a) - F(le0, lp0, b_)) / (2 * h))
            out.append(row)
    return np.asarray(out)


@pytest.mark.parametrize("make,lam", [
    (lambda: synth.circle_se2(), 0.0),
    (lambda: synth.walk_se3(batch=1, n_poses=8, n_loops=4), 1e-3),
])
def test_implicit_gradient_matches_stopped_newton_fd(make, lam):
    p = make()
    g = S.graphs_of(p)[0]
    res = S.solve_graph(g, 6, lam)
    assert res.status == S.OK
    v = torch.as_tensor(rng.normal(size=(g.n_pose, g.G.dof)), dtype=DT)
    gr = S.implicit_grad_graph(g, res, v)
    for key in ["edge_logw", "prior_logw", "tau"]:
        fd = _fd_stopped_newton(g, res, v, key)
        ours = gr[key].numpy()
        scale = max(1e-3, np.abs(fd).max())
        assert np.abs(ours - fd).max() < 1e-6 * scale, key


def test_implicit_gradient_ba_obs_weights_fd():
    p = _small_ba()
    p["obs_w"] = np.exp(rng.normal(scale=0.3, size=len(p["obs_w"])))
    g = S.graphs_of(p)[0]
    g.w_o = torch.as_tensor(p["obs_w"], dtype=DT)
    res = S.solve_graph(g, 5, 1e-3)
    assert res.status == S.OK
    v = torch.as_tensor(rng.normal(size=(g.n_pose, 6)), dtype=DT)
    vq = torch.as_tensor(rng.normal(size=(g.pts.shape[0], 3)), dtype=DT)
    ours = S.implicit_grad_graph(g, res, v, vq)["obs_w"].numpy()
    # the Huber branch switches: make sure both branches occur in this test
    lin = S.linearize_ba(g, res.X, res.pts)
    assert bool((lin.extra["drho"] < 1).any()) and bool((lin.extra["drho"] == 1).any())
    L, Ci, EC = res.factor

    def F(w):
        li = S.linearize_ba(g, res.X, res.pts, w_o=w)
        xc, xp = S.schur_solve(res.lin, L, Ci, EC, li.g, li.gp)   # H frozen at theta_K
        return float(-((v.reshape(-1) * xc).sum() + (vq * xp).sum()))

    h = 1e-6
    fd = []
    for k in range(len(g.w_o)):
        a, b_ = g.w_o.clone(), g.w_o.clone()
        a[k] += h
        b_[k] -= h
        fd.append((F(a) - F(b_)) / (2 * h))
    fd = np.asarray(fd)
    assert np.abs(ours - fd).max() < 1e-6 * np.abs(fd).max()
    # the per-observation Huber radius (the paper's learned BA kernel radius):
    # zero for observations inside the quadratic branch
    od = S.implicit_grad_graph(g, res, v, vq)["obs_delta"].numpy()
    dl0 = torch.full((len(g.oc),), float(g.delta), dtype=DT)

    def Fd(dl):
        li = S.linearize_ba(g, res.X, res.pts, delta_o=dl)
        xc, xp = S.schur_solve(res.lin, L, Ci, EC, li.g, li.gp)
        return float(-((v.reshape(-1) * xc).sum() + (vq * xp).sum()))

    fdd = []
    for k in range(len(g.oc)):
        a, b_ = dl0.clone(), dl0.clone()
        a[k] += h
        b_[k] -= h
        fdd.append((Fd(a) - Fd(b_)) / (2 * h))
    fdd = np.asarray(fdd)
    inside = (lin.extra["drho"] == 1).numpy()
    assert np.all(od[inside] == 0) and np.abs(od[~inside]).max() > 0
    assert np.abs(od - fdd).max() < 1e-6 * np.abs(fdd).max()


def test_implicit_gradient_noiseless_resolve_fd():
    """Noiseless graph: theta* = ground truth, r = 0, so the Gauss-Newton Hessian
    is the exact Hessian and Prop. 1 is the exact derivative of the re-solved
    problem.  Loss L = sum_k <a_k, Log(X_gt,k^-1 X_k)>."""
    p = synth.walk_se3(batch=1, n_poses=8, n_loops=5, noiseless=True)
    G = lie.SE3
    a = torch.as_tensor(rng.normal(size=(8, 6)), dtype=DT)
    Xgt = G.from_storage(torch.as_tensor(p["poses_gt"]))

    def loss(X):
        return float((a * G.log(G.inv(Xgt) @ X)).sum())

    g = S.graphs_of(p, poses=p["poses_gt"])[0]
    res = S.solve_graph(g, 3, 0.0)
    v = (G.jr_inv(G.log(G.inv(Xgt) @ res.X)).transpose(-1, -2) @ a[..., None])[..., 0]
    ours = S.implicit_grad_graph(g, res, v)["tau"].numpy()
    h = 1e-6
    for k in [0, 3, 9]:
        for j in range(6):
            tp = torch.zeros(len(g.ei), 6, dtype=DT)
            tm = tp.clone()
            tp[k, j], tm[k, j] = h, -h
            fp = loss(S.solve_graph(g, 8, 0.0, tau=tp).X)
            fm = loss(S.solve_graph(g, 8, 0.0, tau=tm).X)
            assert abs((fp - fm) / (2 * h) - ours[k, j]) < 1e-6 * max(1.0, np.abs(ours).max())


def test_failed_graph_is_frozen_with_zero_gradient():
    """Without the gauge prior and with lambda = 0 the Hessian is singular: the
    graph keeps its initial poses and gets zero gradients."""
    p = synth.walk_se3(batch=2, n_poses=8, n_loops=4)
    gs = S.graphs_of(p)
    g = gs[1]
    g.pv = g.pv[:0]
    g.PZ = g.PZ[:0]
    g.logw_p = g.logw_p[:0]
    res = S.solve_graph(g, 4, 0.0)
    assert res.status == S.NOT_PD
    assert torch.equal(res.X, g.X)
    assert len(set(res.objective)) == 1 and len(res.objective) == 5
    gr = S.implicit_grad_graph(g, res, torch.ones(8, 6, dtype=DT))
    assert float(gr["tau"].abs().max()) == 0.0


def test_sparse_assembly_equals_dense():
    p = synth.lattice_se3(batch=1, side=3)
    g = S.graphs_of(p)[0]
    lin = S.linearize_pose_graph(g, g.X)
    s, H, gv = S.linearize_pose_graph_sparse(g, g.X)
    assert abs(s - float(lin.S)) < 1e-12 * max(1.0, s)
    assert np.abs(H.toarray() - lin.H.numpy()).max() < 1e-12 * np.abs(H.toarray()).max()
    assert np.abs(gv - lin.g.numpy()).max() < 1e-12 * np.abs(gv).max()


def test_unrolled_gradient_approaches_gn_implicit_linearly_in_noise():
    """Reading of Prop. 1 (Gauss-Newton Hessian in the stopped slot): the
    unrolled gradient (autograd through K converged Gauss-Newton steps)
    tends to the exact implicit derivative, which differs from the
    Gauss-Newton implicit gradient by a term proportional to the residual.
    With the measurement noise scaled by 1, 0.1 and 0.01 the relative gap
    must shrink linearly (measured 1.6e-2, 1.6e-3, 1.6e-4)."""
    import dataclasses
    from oracle import lie

    def gap(scale, K=25):
        p = synth.walk_se3(batch=1, n_poses=12, n_loops=6, sigma_t=0.05 * scale, sigma_r=0.01 * scale, seed=3)
        g = S.graphs_of(p)[0]
        logw = g.logw_e.clone().requires_grad_(True)
        tau = torch.zeros(g.ei.shape[0], 6, dtype=torch.float64, requires_grad=True)
        r = S.solve_graph(dataclasses.replace(g, logw_e=logw, tau=tau), K, 0.0)
        Xg = lie.SE3.from_storage(torch.as_tensor(p["poses_gt"]))
        L = (lie.SE3.log(lie.SE3.inv(Xg) @ r.X) ** 2).sum()
        gw, gt = torch.autograd.grad(L, [logw, tau])
        r0 = S.solve_graph(g, K, 0.0)
        _, v = S.pose_error_loss_and_seed("SE3", lie.SE3.to_storage(r0.X).numpy(), p["poses_gt"])
        gi = S.implicit_grad_graph(g, r0, torch.as_tensor(v))
        a = torch.cat([gw, gt.reshape(-1)])
        b = torch.cat([gi["edge_logw"].detach(), gi["tau"].detach().reshape(-1)])
        return float((a - b).norm() / b.norm())

    g1, g2, g3 = gap(1.0), gap(0.1), gap(0.01)
    assert 1e-3 < g1 < 0.1
    assert 0.05 < g2 / g1 < 0.2 and 0.05 < g3 / g2 < 0.2


def _single_pose_rotation_problem(group, theta0):
    """One pose, only its prior, off by a pure rotation theta0 about z."""
    G = lie.group(group)
    d = G.dof
    P = G.exp(torch.as_tensor(np.array([[0.3, -0.2, 0.1, 0.05, -0.1, 0.2][:d]]), dtype=torch.float64))
    rot = np.zeros((1, d))
    rot[0, d - 1] = theta0
    X0 = P @ G.exp(torch.as_tensor(rot, dtype=torch.float64))
    store = lambda X: G.to_storage(X).numpy()
    return {
        "group": group, "pose_off": np.array([0, 1], np.int32), "poses_init": store(X0), "poses_gt": store(P),
        "edge_off": np.array([0, 0], np.int32), "edge_ij": np.zeros((0, 2), np.int32),
        "edge_meas": store(P)[:0], "edge_logw": np.zeros(0),
        "prior_off": np.array([0, 1], np.int32), "prior_var": np.array([0], np.int32),
        "prior_meas": store(P), "prior_logw": np.zeros(1),
    }


@pytest.mark.parametrize("group", ["SE2", "SE3"])
def test_adaptive_lm_closed_form_single_pose(group):
    """Adaptive damping on one pose with a pure-rotation prior error theta:
    the Jacobian is block diagonal with a unit rotation block, so the damped
    step is theta / (1 + lambda), every step decreases S = theta^2 / 2 and is
    kept, lambda is divided by 10 each time (floor 1e-7), and
    theta_K = theta_0 prod_t lambda_t / (1 + lambda_t)."""
    theta0, lam0, K = 0.7, 1.0, 9
    p = _single_pose_rotation_problem(group, theta0)
    g = S.graphs_of(p)[0]
    r = S.solve_graph(g, K, lam0, adaptive=True)
    lams, theta = [], theta0
    lam = lam0
    for _ in range(K):
        lams.append(lam)
        theta *= lam / (1.0 + lam)
        lam = max(lam / 10.0, 1e-7)
    assert r.lambdas == pytest.approx(lams, rel=1e-15)
    G = lie.group(group)
    err = G.log(G.inv(g.PZ[0]) @ r.X[0])
    expect = np.zeros(G.dof)
    expect[-1] = theta
    assert np.abs(err.numpy() - expect).max() < 1e-12 * theta0
    assert r.objective[-1] == pytest.approx(0.5 * theta ** 2, rel=1e-10)


def test_adaptive_lm_rejects_and_recovers():
    """SE(2) circle from a poor initial guess: the first two damped steps
    increase the objective and are rejected (theta kept, objective repeated,
    lambda x 10); afterwards steps are kept (lambda / 10).  The objective
    sequence never increases, and each repeat coincides with a x10."""
    p = synth.circle_se2(batch=1, seed=3)
    g = S.graphs_of(p)[0]
    rng = np.random.default_rng(13)
    xi = torch.zeros(g.X.shape[0], 3, dtype=torch.float64)
    xi[:, 2] = torch.as_tensor(rng.normal(scale=1.6, size=g.X.shape[0]))
    xi[:, :2] = torch.as_tensor(rng.normal(scale=1.6, size=(g.X.shape[0], 2)))
    g.X = lie.SE2.retract(g.X, xi)
    K = 8
    r = S.solve_graph(g, K, 1e-4, adaptive=True)
    ob, lams = r.objective, r.lambdas
    assert all(ob[t + 1] <= ob[t] for t in range(K))
    rejected = [ob[t + 1] == ob[t] for t in range(K - 1)]
    assert rejected[:2] == [True, True] and not any(rejected[2:5])
    for t in range(K - 1):
        assert lams[t + 1] == (min(lams[t] * 10.0, 1e7) if rejected[t] else max(lams[t] / 10.0, 1e-7))


# ---------------------------------------------------------------------------
# Direct loss minimisation (Section 4.3, Appendix G)
# ---------------------------------------------------------------------------
def _converged_walk(seed=5):
    p = synth.walk_se3(batch=1, n_poses=10, n_loops=5, seed=seed)
    g = S.graphs_of(p)[0]
    tau0 = torch.as_tensor(rng.normal(scale=0.01, size=(len(g.ei), 6)), dtype=DT)
    import dataclasses
    g = dataclasses.replace(g, tau=tau0)
    res = S.solve_graph(g, 12, 0.0)
    assert res.status == S.OK and float(res.lin.g.abs().max()) < 1e-12
    return g, res


def test_dlm_gradient_tends_linearly_to_implicit():
    """The DLM estimate differs from the implicit gradient (pinned above by
    finite differences of the stopped Newton step) by a term linear in eps:
    the relative gap must fall tenfold per decade of eps."""
    g, res = _converged_walk()
    v = torch.as_tensor(rng.normal(size=(g.n_pose, 6)), dtype=DT)
    gi = S.implicit_grad_graph(g, res, v)
    ref = torch.cat([gi["edge_logw"], gi["prior_logw"], gi["tau"].reshape(-1)])

    def gap(eps):
        gd = S.dlm_grad_graph(g, res, v, eps)
        ours = torch.cat([gd["edge_logw"], gd["prior_logw"], gd["tau"].reshape(-1)])
        return float((ours - ref).norm() / ref.norm())

    g3, g4, g5 = gap(1e-3), gap(1e-4), gap(1e-5)
    assert g3 < 0.5
    assert 0.07 < g4 / g3 < 0.13 and 0.07 < g5 / g4 < 0.13


def test_dlm_step_minimises_regularised_gauss_newton_model():
    """theta_direct = theta_K Exp(delta) with delta the minimiser of
    1/2 ||r + J delta||^2 + ||eps delta - v/2||^2, J the Jacobian of the
    weighted residual vector r under right perturbations; J is taken here by
    central differences of the costs, independently of the oracle's
    analytic Jacobians, and eps is large so that the 2 eps^2 damping
    matters."""
    g, res = _converged_walk(seed=6)
    d, N = 6, g.n_pose
    v = torch.as_tensor(rng.normal(size=(N, d)), dtype=DT)
    eps = 0.7

    def rvec(X):
        k = S.pose_costs(g, X, g.tau)
        return torch.cat([(k["w_e"][:, None] * k["c_e"]).reshape(-1), (k["w_p"][:, None] * k["c_p"]).reshape(-1)])

    r0 = rvec(res.X)
    h = 1e-6
    cols = []
    for q in range(N * d):
        e = torch.zeros(N * d, dtype=DT)
        e[q] = h
        cols.append((rvec(g.G.retract(res.X, e.reshape(N, d))) - rvec(g.G.retract(res.X, -e.reshape(N, d)))) / (2 * h))
    J = torch.stack(cols, 1).numpy()
    A = np.vstack([J, np.sqrt(2.0) * eps * np.eye(N * d)])
    rhs = np.concatenate([-r0.numpy(), v.reshape(-1).numpy() / np.sqrt(2.0)])
    want = np.linalg.lstsq(A, rhs, rcond=None)[0]
    got = S.dlm_grad_graph(g, res, v, eps)["delta"].reshape(-1).numpy()
    assert np.abs(got - want).max() < 1e-6 * np.abs(want).max()


def test_dlm_ba_gradient_tends_linearly_to_implicit():
    """Bundle adjustment: the DLM estimate for the observation weights and
    prior log-weights approaches the implicit gradient (pinned above by
    finite differences) linearly in eps, with camera and point seeds.  The
    Huber reweighting converges linearly, so the solve runs to |g| ~ 1e-9
    (DLM takes theta_K as a stationary point; a residual gradient adds a
    |g| / eps term)."""
    p = _small_ba()
    g = S.graphs_of(p)[0]
    res = S.solve_graph(g, 100, 0.0)
    assert float(res.lin.g.norm()) < 1e-8
    vc = torch.as_tensor(rng.normal(size=(g.X.shape[0], 6)), dtype=DT)
    vp = torch.as_tensor(rng.normal(size=(g.pts.shape[0], 3)), dtype=DT)
    gi = S.implicit_grad_graph(g, res, vc, vp)
    ref = torch.cat([gi["obs_w"], gi["prior_logw"], gi["obs_delta"]])

    def gap(eps):
        gd = S.dlm_grad_ba(g, res, vc, vp, eps)
        return float((torch.cat([gd["obs_w"], gd["prior_logw"], gd["obs_delta"]]) - ref).norm() / ref.norm())

    g2, g3, g4 = gap(1e-2), gap(1e-3), gap(1e-4)
    assert g2 < 0.05
    assert 0.07 < g3 / g2 < 0.13 and 0.07 < g4 / g3 < 0.13


def test_dlm_ba_step_is_the_schur_solution_of_the_regularised_system():
    """The DLM step over cameras and points equals the oracle's Schur solve
    of the same system (H* + 2 eps^2 I, right-hand side -g* + eps v), a
    different route than the full-system solve the DLM gradient uses."""
    p = _small_ba()
    g = S.graphs_of(p)[0]
    res = S.solve_graph(g, 6, 1e-3)
    vc = rng.normal(size=(g.X.shape[0], 6))
    vp = rng.normal(size=(g.pts.shape[0], 3))
    eps = 0.5
    gd = S.dlm_grad_ba(g, res, vc, vp, eps)
    lin = res.lin
    L, Ci, EC = S.schur_factor(lin, 2.0 * eps * eps)
    dc, dp = S.schur_solve(lin, L, Ci, EC, -lin.g + eps * torch.as_tensor(vc.reshape(-1)),
                           -lin.gp + eps * torch.as_tensor(vp))
    ref = torch.cat([dc, dp.reshape(-1)])
    assert float((gd["delta"] - ref).norm() / ref.norm()) < 1e-10


def test_dlm_failed_graph_gets_zero_gradient():
    p = synth.walk_se3(batch=1, n_poses=6, n_loops=2, seed=7)
    g = S.graphs_of(p)[0]
    res = S.solve_graph(g, 3, 0.0)
    res.status = S.NOT_PD
    gd = S.dlm_grad_graph(g, res, torch.ones(g.n_pose, 6, dtype=DT), 1e-3)
    assert all(float(t.abs().max()) == 0.0 for t in (gd["edge_logw"], gd["prior_logw"], gd["tau"]))


# ---------------------------------------------------------------------------
# Exact-Hessian implicit gradient against the re-solved optimum
# ---------------------------------------------------------------------------
def test_exact_implicit_gradient_matches_resolved_optimum_fd():
    """With noisy measurements (non-zero residuals at the optimum) the exact
    implicit gradient equals central differences of the fully re-solved
    optimum, L(phi) = sum_k v_k . Log(X_k*^-1 X_k*(phi)) (its tangent gradient
    at phi is v), to 1e-6, while the Gauss-Newton implicit gradient misses by
    the residual term (more than 1e-3 here)."""
    import dataclasses
    p = synth.walk_se3(batch=1, n_poses=8, n_loops=4, sigma_t=0.1, sigma_r=0.03, seed=9)
    g = S.graphs_of(p)[0]
    g = dataclasses.replace(g, tau=torch.zeros(len(g.ei), 6, dtype=DT))
    base = S.solve_graph(g, 25, 0.0)
    assert base.status == S.OK and float(base.lin.g.abs().max()) < 1e-12
    G = g.G
    v = torch.as_tensor(rng.normal(size=(g.n_pose, 6)), dtype=DT)
    ex = S.exact_implicit_grad_graph(g, base, v)
    gn = S.implicit_grad_graph(g, base, v)

    def F(le, tau):
        r = S.solve_graph(dataclasses.replace(g, X=base.X, logw_e=le, tau=tau), 12, 0.0)
        return float((G.log(G.inv(base.X) @ r.X) * v).sum())

    h = 1e-5
    le0, t0 = g.logw_e.clone(), g.tau.clone()
    fd, ours, theirs = [], [], []
    for k in (0, 3, 7, 9):
        a, b_ = le0.clone(), le0.clone()
        a[k] += h
        b_[k] -= h
        fd.append((F(a, t0) - F(b_, t0)) / (2 * h))
        ours.append(float(ex["edge_logw"][k]))
        theirs.append(float(gn["edge_logw"][k]))
    for k, j in ((1, 0), (5, 4), (10, 2)):
        a, b_ = t0.clone(), t0.clone()
        a[k, j] += h
        b_[k, j] -= h
        fd.append((F(le0, a) - F(le0, b_)) / (2 * h))
        ours.append(float(ex["tau"][k, j]))
        theirs.append(float(gn["tau"][k, j]))
    fd, ours, theirs = map(np.asarray, (fd, ours, theirs))
    scale = np.abs(fd).max()
    assert np.abs(ours - fd).max() < 1e-6 * scale
    assert np.abs(theirs - fd).max() > 1e-3 * scale


def test_exact_hessian_equals_gauss_newton_at_zero_residual():
    """Noiseless measurements: every residual vanishes at the ground truth,
    so the second-order terms vanish and the two Hessians (hence the two
    gradients) agree."""
    p = synth.walk_se3(batch=1, n_poses=6, n_loops=3, sigma_t=0.0, sigma_r=0.0, seed=4)
    g = S.graphs_of(p)[0]
    res = S.solve_graph(g, 4, 0.0)
    Hx = S.exact_hessian_graph(g, res.X)
    assert float((Hx - res.lin.H).abs().max()) < 1e-9 * float(res.lin.H.abs().max())


# ---------------------------------------------------------------------------
# Dogleg (trust region)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("group", ["SE2", "SE3"])
def test_dogleg_closed_form_single_pose(group):
    """One pose, a pure-rotation prior error theta: g = c, H acts as the
    identity along c, so the Gauss-Newton and Cauchy points coincide at the
    target.  While theta > radius the step is the scaled gradient of length
    radius (rho = 1 on the boundary: the radius doubles); once theta <= radius
    the Gauss-Newton step lands on the target (inside: the radius stays).
    theta 1.0 with radius 0.1: theta = 1.0, 0.9, 0.7, 0.3, 0 and radii 0.1,
    0.2, 0.4, 0.8."""
    p = _single_pose_rotation_problem(group, 1.0)
    g = S.graphs_of(p)[0]
    r = S.solve_graph(g, 4, 0.0, dogleg_radius=0.1)
    assert r.radii == pytest.approx([0.1, 0.2, 0.4, 0.8], rel=1e-12)
    assert r.objective == pytest.approx([0.5, 0.405, 0.245, 0.045, 0.0], rel=1e-10, abs=1e-20)


def test_dogleg_with_huge_radius_is_gauss_newton():
    """Every Gauss-Newton point lies inside the region: the first steps are
    the Gauss-Newton steps exactly until the rounding floor, where Gauss-Newton
    lets S rise by an ulp and the dogleg refuses such a step."""
    p = synth.walk_se3(batch=1, n_poses=12, n_loops=8, seed=21)
    g = S.graphs_of(p)[0]
    a = S.solve_graph(g, 5, 0.0)
    b = S.solve_graph(g, 5, 0.0, dogleg_radius=1e6)
    assert torch.equal(a.X, b.X) and a.objective == b.objective
    b = S.solve_graph(g, 8, 0.0, dogleg_radius=1e6)
    assert all(y <= x for x, y in zip(b.objective, b.objective[1:]))


def test_dogleg_monotone_and_shrinks_on_rejection():
    """From a poor initial guess: the objective never increases, every
    rejected step (repeated objective) shrinks the radius to a quarter of the
    step length, and some steps are rejected and some land on the boundary."""
    p = synth.walk_se3(batch=1, n_poses=16, n_loops=10, seed=22, init_noise=(0.6, 0.4))
    g = S.graphs_of(p)[0]
    r = S.solve_graph(g, 12, 0.0, dogleg_radius=2.0)
    ob = r.objective
    assert all(b <= a for a, b in zip(ob, ob[1:]))
    rej = [t for t in range(12) if ob[t + 1] == ob[t]]
    assert rej, "expected at least one rejected step"
    for t in rej:
        if t + 1 < 12:
            assert r.radii[t + 1] < r.radii[t]


# ---------------------------------------------------------------------------
# Unrolled and truncated gradients
# ---------------------------------------------------------------------------
def test_unrolled_gradient_matches_fd_of_the_k_step_map():
    """The unrolled gradient is the exact derivative of the K-step map:
    central differences of F(phi) = sum_p v_p . Log(theta_K^-1 theta_K(phi))
    (K = 3 LM steps from the same start) agree to 1e-7; truncation to the
    last 3 steps equals full unrolling, and its adjoint at theta_0 matches
    differences in the initial poses."""
    import dataclasses
    p = synth.walk_se3(batch=1, n_poses=8, n_loops=4, sigma_t=0.1, sigma_r=0.03, seed=12)
    g = S.graphs_of(p)[0]
    g = dataclasses.replace(g, tau=torch.as_tensor(rng.normal(scale=0.01, size=(len(g.ei), 6)), dtype=DT))
    K, lam = 3, 1e-2
    v = torch.as_tensor(rng.normal(size=(g.n_pose, 6)), dtype=DT)
    un = S.unrolled_grad_graph(g, K, lam, v)
    tr = S.unrolled_grad_graph(g, K, lam, v, steps=K)
    for k in ("edge_logw", "prior_logw", "tau", "adjoint"):
        assert torch.equal(un[k], tr[k]), k
    G = g.G
    XK = S.solve_graph(g, K, lam).X

    def F(**kw):
        r = S.solve_graph(dataclasses.replace(g, **kw), K, lam)
        return float((G.log(G.inv(XK) @ r.X) * v).sum())

    h = 1e-6
    fd, ours = [], []
    for k in (0, 4, 9):
        a, b_ = g.logw_e.clone(), g.logw_e.clone()
        a[k] += h
        b_[k] -= h
        fd.append((F(logw_e=a) - F(logw_e=b_)) / (2 * h))
        ours.append(float(un["edge_logw"][k]))
    for k, j in ((2, 1), (7, 5)):
        a, b_ = g.tau.clone(), g.tau.clone()
        a[k, j] += h
        b_[k, j] -= h
        fd.append((F(tau=a) - F(tau=b_)) / (2 * h))
        ours.append(float(un["tau"][k, j]))
    for q, j in ((3, 0), (5, 4)):
        e = torch.zeros(g.n_pose, 6, dtype=DT)
        e[q, j] = h
        fd.append((F(X=G.retract(g.X, e)) - F(X=G.retract(g.X, -e))) / (2 * h))
        ours.append(float(un["adjoint"][q, j]))
    fd, ours = np.asarray(fd), np.asarray(ours)
    assert np.abs(ours - fd).max() < 1e-7 * np.abs(fd).max()


def test_truncated_gradient_is_the_last_steps_only():
    """Truncation to T steps equals full unrolling of a problem that starts at
    theta_{K-T}."""
    import dataclasses
    p = synth.walk_se3(batch=1, n_poses=8, n_loops=4, seed=13)
    g = S.graphs_of(p)[0]
    K, T, lam = 5, 2, 1e-3
    v = torch.as_tensor(rng.normal(size=(g.n_pose, 6)), dtype=DT)
    tr = S.unrolled_grad_graph(g, K, lam, v, steps=T)
    mid = S.solve_graph(g, K - T, lam).X
    un = S.unrolled_grad_graph(dataclasses.replace(g, X=mid), T, lam, v)
    for k in ("edge_logw", "prior_logw", "tau"):
        assert torch.allclose(tr[k], un[k], rtol=1e-12, atol=1e-14), k


# ---------------------------------------------------------------------------
# Welsch robust loss with a learnable radius
# ---------------------------------------------------------------------------
def test_welsch_definition():
    s = torch.tensor([0.0, 1e-6, 0.3, 4.0, 50.0], dtype=DT)
    logc = torch.full_like(s, np.log(1.5))
    rho, drho = S.welsch(s, logc)
    c2 = 2.25
    assert torch.allclose(rho, c2 * (1 - torch.exp(-s / c2)), rtol=1e-15)
    assert float(rho[0]) == 0.0 and float(drho[0]) == 1.0
    assert abs(float(rho[1]) - 1e-6) < 1e-12                    # rho ~ s for s << c^2
    assert abs(float(rho[4]) - c2) < 1e-8                       # rho -> c^2 for s >> c^2
    ds = 1e-7
    fd = (S.welsch(s + ds, logc)[0] - S.welsch(s - ds, logc)[0]) / (2 * ds)
    assert torch.allclose(fd[1:], drho[1:], rtol=1e-6)


def test_welsch_huge_radius_is_least_squares():
    import dataclasses
    p = synth.walk_se3(batch=1, n_poses=10, n_loops=6, seed=31)
    g = S.graphs_of(p)[0]
    gr = dataclasses.replace(g, logc_e=torch.full((len(g.ei),), 30.0, dtype=DT))
    a, b = S.solve_graph(g, 5, 1e-3), S.solve_graph(gr, 5, 1e-3)
    assert float((a.X - b.X).abs().max()) < 1e-12
    v = torch.as_tensor(rng.normal(size=(g.n_pose, 6)), dtype=DT)
    ga, gb = S.implicit_grad_graph(g, a, v), S.implicit_grad_graph(gr, b, v)
    assert torch.allclose(ga["edge_logw"], gb["edge_logw"], rtol=1e-9, atol=1e-12)
    assert float(gb["edge_logc"].abs().max()) < 1e-12


def test_welsch_implicit_gradient_matches_stopped_newton_fd():
    """Proposition 1 with the reweighted Gauss-Newton Hessian in the stopped
    slot: central differences of F(phi) = -v^T Hbar^-1 g(theta_K; phi), Hbar
    frozen, in the Welsch log-radii and log-weights of a walk with outliers."""
    import dataclasses
    p = synth.walk_se3(batch=1, n_poses=10, n_loops=6, seed=32, outliers=2)
    g = S.graphs_of(p)[0]
    g = dataclasses.replace(g, logc_e=torch.as_tensor(rng.normal(np.log(0.5), 0.3, size=len(g.ei)), dtype=DT))
    res = S.solve_graph(g, 8, 1e-3)
    assert res.status == S.OK
    (L,) = res.factor
    v = torch.as_tensor(rng.normal(size=(g.n_pose, 6)), dtype=DT)
    gr = S.implicit_grad_graph(g, res, v)

    def F(lc, le):
        lin = S.linearize_pose_graph(g, res.X, logw_e=le, logc_e=lc)
        return float(-(v.reshape(-1) * torch.cholesky_solve(lin.g[:, None], L)[:, 0]).sum())

    h = 1e-6
    lc0, le0 = g.logc_e.clone(), g.logw_e.clone()
    fd_c, fd_w = [], []
    for k in range(len(lc0)):
        a, b_ = lc0.clone(), lc0.clone()
        a[k] += h
        b_[k] -= h
        fd_c.append((F(a, le0) - F(b_, le0)) / (2 * h))
        a, b_ = le0.clone(), le0.clone()
        a[k] += h
        b_[k] -= h
        fd_w.append((F(lc0, a) - F(lc0, b_)) / (2 * h))
    # central differences with h = 1e-6 carry ~1e-9 of rounding noise on these gradients (~5e-4)
    for fd, ours in ((np.asarray(fd_c), gr["edge_logc"].numpy()), (np.asarray(fd_w), gr["edge_logw"].numpy())):
        assert np.abs(ours - fd).max() < 1e-5 * max(1e-3, np.abs(fd).max())
    assert np.abs(fd_c).max() > 1e-5


def test_welsch_rejects_outliers():
    """Four gross loop-closure outliers: plain least squares is dragged away
    from the ground truth (max pose error ~9), a Welsch radius of 0.5 stays at
    the level of the odometry drift (~0.27, the initial guess has 0.33)."""
    import dataclasses
    from oracle import lie
    p = synth.walk_se3(batch=1, n_poses=16, n_loops=12, seed=33, outliers=4)
    g = S.graphs_of(p)[0]
    Xg = lie.SE3.from_storage(torch.as_tensor(p["poses_gt"]))
    err = lambda X: float(lie.SE3.log(lie.SE3.inv(Xg) @ X).norm(dim=-1).max())
    plain = S.solve_graph(g, 10, 1e-3)
    rob = S.solve_graph(dataclasses.replace(g, logc_e=torch.full((len(g.ei),), np.log(0.5), dtype=DT)), 10, 1e-3)
    assert err(rob.X) < 0.5 and err(plain.X) > 10 * err(rob.X)


@pytest.mark.parametrize("lam,with_tau", [(0.0, False), (1e-3, True)])
def test_sparse_oracle_equals_dense_oracle(lam, with_tau):
    """The sparse-factorisation oracle (for graphs whose dense H does not fit)
    takes the same steps as the dense one: iterates, objectives and the
    implicit gradient agree on a small lattice with long-range edges."""
    p = synth.lattice_se3(batch=1, side=4, seed=6)
    g = S.graphs_of(p)[0]
    if with_tau:
        g.tau = torch.as_tensor(0.01 * np.random.default_rng(2).normal(size=(len(g.ei), 6)), dtype=torch.float64)
    a = S.solve_graph(g, 4, lam)
    b = S.solve_graph_sparse(g, 4, lam)
    assert a.status == b.status == S.OK
    assert float((lie.SE3.to_storage(a.X) - lie.SE3.to_storage(b.X)).abs().max()) < 1e-12
    assert np.allclose(a.objective, b.objective, rtol=1e-12, atol=0)
    _, v = S.pose_error_loss_and_seed("SE3", lie.SE3.to_storage(a.X).numpy(), p["poses_gt"])
    ga = S.implicit_grad_graph(g, a, torch.as_tensor(v))
    gb = S.implicit_grad_graph_sparse(g, b, v)
    scale = max(float(ga[k].abs().max()) for k in ("edge_logw", "prior_logw", "tau"))
    for k in ("edge_logw", "prior_logw", "tau", "u"):
        ref = ga[k].detach().numpy()
        floor = np.abs(ref).max() if k == "u" else scale
        assert np.abs(gb[k].detach().numpy() - ref).max() < 1e-9 * floor, k


def test_sparse_oracle_flags_a_singular_system():
    """Without the prior the pose graph's H is singular (gauge freedom): the
    sparse oracle reports NOT_PD, keeps theta_0 and gives zero gradients,
    like the dense oracle."""
    p = synth.lattice_se3(batch=1, side=3, seed=1)
    g = S.graphs_of(p)[0]
    g.pv = g.pv[:0]
    g.PZ = g.PZ[:0]
    g.logw_p = g.logw_p[:0]
    a, b = S.solve_graph(g, 3, 0.0), S.solve_graph_sparse(g, 3, 0.0)
    assert a.status == b.status == S.NOT_PD
    assert torch.equal(b.X, g.X)
    assert b.objective == a.objective
    gr = S.implicit_grad_graph_sparse(g, b, np.ones((g.X.shape[0], 6)))
    assert float(gr["tau"].abs().max()) == 0.0
