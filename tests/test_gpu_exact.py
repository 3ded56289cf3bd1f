"""GPU parity of the exact-Hessian implicit backward (Proposition 1 with the
Hessian of S in place of the Gauss-Newton one) through the C ABI against the
oracle's exact_implicit_grad_graph.

The oracle forms the exact Hessian by torch.autograd and solves it directly;
the GPU applies it matrix-free (dual numbers per cost) inside iterative
refinement preconditioned by the cached Gauss-Newton factor.  With enough
sweeps the two agree to the float64 tolerance of the implicit gradient,
max(1e-10, 0.5 cond(H) eps64) per graph; the oracle is evaluated at the poses
the GPU solve returned, so the test checks the backward alone.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import synth
from oracle import solve as S

from gpu_util import gpu_solve, oracle_graphs, rel, t

pytestmark = pytest.mark.gpu
rng = np.random.default_rng(4411)


def _problem(group, seed):
    if group == "SE3":
        p = synth.uneven_walk_se3(batch=5, n_min=3, n_max=30, seed=seed)
    else:
        p = synth.circle_se2(batch=4, n_poses=20, n_loops=8, seed=seed)
    p["edge_logw"] = rng.normal(scale=0.3, size=len(p["edge_logw"]))
    p["prior_logw"] = rng.normal(scale=0.3, size=len(p["prior_logw"]))
    dof = 6 if group == "SE3" else 3
    tau = 0.01 * rng.normal(size=(len(p["edge_logw"]), dof))
    return p, tau


def _run(plan, poses, status, dev, seed, mode, sweeps=0):
    out = plan.backward(poses, dev["edge_meas"], dev["edge_logw"], dev["prior_meas"], dev["prior_logw"],
                        status, t(seed), edge_tau=dev["edge_tau"], want_adjoint=True, mode=mode, sweeps=sweeps)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _errors(p, tau, plan, poses, status, dev, seed, gr, graphs):
    """Per graph: (gradient error, adjoint error, tolerance) against the
    oracle's exact gradient at the GPU's theta_K."""
    X = poses.cpu()
    gs = oracle_graphs(p, tau, graphs)
    out = []
    for gi, b in enumerate(graphs):
        g = gs[gi]
        lo, hi = int(p["pose_off"][b]), int(p["pose_off"][b + 1])
        Xb = g.G.from_storage(X[lo:hi])
        res = S.GraphResult(X=Xb, pts=None, objective=[], status=S.OK, lin=S.linearize_pose_graph(g, Xb, tau=g.tau))
        ref = S.exact_implicit_grad_graph(g, res, torch.as_tensor(seed[lo:hi]))
        e0, e1 = int(p["edge_off"][b]), int(p["edge_off"][b + 1])
        q0, q1 = int(p["prior_off"][b]), int(p["prior_off"][b + 1])
        mine = np.concatenate([gr["edge_logw"][e0:e1], gr["edge_tau"][e0:e1].ravel(), gr["prior_logw"][q0:q1]])
        theirs = np.concatenate([ref["edge_logw"].numpy(), ref["tau"].numpy().ravel(), ref["prior_logw"].numpy()])
        ev = np.linalg.eigvalsh(res.lin.H.numpy())
        tol = max(1e-10, 0.5 * (ev[-1] / ev[0]) * np.finfo(np.float64).eps)
        out.append((rel(mine, theirs), rel(gr["adjoint"][lo:hi], ref["u"].numpy()), tol))
    return out


@pytest.mark.parametrize("solver", ["dense", "sparse", "sparse-block"])
@pytest.mark.parametrize("group", ["SE2", "SE3"])
def test_exact_backward_matches_oracle_ragged_batch(group, solver):
    p, tau = _problem(group, seed=41)
    plan, poses, objective, status, dev = gpu_solve(p, 10, 1e-3, tau=tau, solver=solver)
    assert (status.cpu().numpy() == S.OK).all()
    seed = rng.normal(size=(int(p["pose_off"][-1]), plan.dof))
    gr = _run(plan, poses, status, dev, seed, "exact", sweeps=30)
    B = len(p["pose_off"]) - 1
    for b, (eg, eu, tol) in enumerate(_errors(p, tau, plan, poses, status, dev, seed, gr, list(range(B)))):
        print(f"\n[exact {group} {solver}] graph {b}: gradient {eg:.2e} adjoint {eu:.2e} tolerance {tol:.2e}")
        assert eg < tol and eu < tol, (b, eg, eu, tol)


@pytest.mark.parametrize("solver", ["dense", "sparse"])
def test_exact_backward_converges_geometrically_and_zero_sweeps_is_gauss_newton(solver):
    """Sweeps = 0 reproduces the Gauss-Newton implicit backward; the error
    against the oracle's exact gradient then shrinks by about the same factor
    per sweep (the spectral radius of I - H*^-1 Hx)."""
    p = synth.walk_se3(batch=2, n_poses=24, n_loops=16, sigma_t=0.1, sigma_r=0.03, seed=8)
    plan, poses, objective, status, dev = gpu_solve(p, 12, 0.0, solver=solver)
    seed = rng.normal(size=(int(p["pose_off"][-1]), 6))
    imp = _run(plan, poses, status, dev, seed, "implicit")
    ex0 = _run(plan, poses, status, dev, seed, "exact", sweeps=0)
    for k in ("edge_logw", "edge_tau", "prior_logw", "adjoint"):
        assert np.array_equal(imp[k], ex0[k]), k
    errs = []
    for s in (0, 1, 2, 3):
        gr = _run(plan, poses, status, dev, seed, "exact", sweeps=s)
        errs.append(max(e[0] for e in _errors(p, None, plan, poses, status, dev, seed, gr, [0, 1])))
    print("\n[exact] error per sweep count", " ".join(f"{e:.2e}" for e in errs))
    assert errs[0] > 1e-4
    for a, b in zip(errs, errs[1:]):
        assert b < 0.3 * a


def test_exact_backward_walk64_b128_sampled_graphs():
    p = synth.walk_se3(batch=128)
    plan, poses, objective, status, dev = gpu_solve(p, 10, 1e-3)
    seed = rng.normal(size=(int(p["pose_off"][-1]), 6))
    gr = _run(plan, poses, status, dev, seed, "exact", sweeps=12)
    for eg, eu, tol in _errors(p, None, plan, poses, status, dev, seed, gr, [0, 37, 81, 127]):
        assert eg < tol and eu < tol, (eg, eu, tol)


def test_exact_backward_failed_graphs_and_argument_checks():
    from paper_2207_09442_amd import DnlsError, Plan
    p = synth.walk_se3(batch=2, n_poses=8, n_loops=4, seed=17)
    last = int(p["pose_off"][1]) + 7
    keep = ~((p["edge_ij"][:, 0] == last) | (p["edge_ij"][:, 1] == last))
    counts = [int(keep[p["edge_off"][b]:p["edge_off"][b + 1]].sum()) for b in range(2)]
    p["edge_ij"], p["edge_meas"], p["edge_logw"] = p["edge_ij"][keep], p["edge_meas"][keep], p["edge_logw"][keep]
    p["edge_off"] = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    plan, poses, objective, status, dev = gpu_solve(p, 4, 0.0)
    assert status.cpu().tolist() == [S.OK, S.NOT_PD]
    seed = rng.normal(size=(int(p["pose_off"][-1]), 6))
    gr = _run(plan, poses, status, dev, seed, "exact", sweeps=4)
    e0, lo = int(p["edge_off"][1]), int(p["pose_off"][1])
    assert np.all(gr["edge_logw"][e0:] == 0) and np.all(gr["edge_tau"][e0:] == 0)
    assert np.all(gr["adjoint"][lo:] == 0)
    assert np.all(np.isfinite(gr["edge_logw"][:e0])) and np.abs(gr["edge_logw"][:e0]).max() > 0
    for s in (-1, 65):
        with pytest.raises(DnlsError):
            _run(plan, poses, status, dev, seed, "exact", sweeps=s)
    q = synth.bundle_adjustment(batch=1, n_cams=8, n_points=40, obs_per_point=4, seed=9)
    ba = Plan(q, 2, lam=1e-3, solver="schur", device="cuda")
    cams, pts = t(q["poses_init"]), t(q["points_init"])
    aux = dict(obs_uv=t(q["obs_uv"]), obs_w=t(q["obs_w"]), prior_meas=t(q["prior_meas"]),
               prior_logw=t(q["prior_logw"]))
    _, stb = ba.solve_ba(cams, pts, **aux)
    from paper_2207_09442_amd import _BackwardArgs, _check, _ptr, _stream, lib
    import ctypes
    args = _BackwardArgs()
    args.poses, args.points = _ptr(cams), _ptr(pts)
    args.obs_uv, args.obs_w = _ptr(aux["obs_uv"]), _ptr(aux["obs_w"])
    args.prior_meas, args.prior_logw = _ptr(aux["prior_meas"]), _ptr(aux["prior_logw"])
    args.status, args.factor, args.workspace = _ptr(stb), ba._aligned(ba.factor), ba._aligned(ba.workspace)
    args.seed_pose = _ptr(t(np.zeros((8, 6))))
    args.mode, args.sweeps = 2, 4
    with pytest.raises(DnlsError):
        _check(lib().dnls_backward(ba._h, ctypes.byref(args), _stream()), "dnls_backward")
