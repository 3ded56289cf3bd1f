"""GPU parity of the Welsch robust loss on pose-graph edges (learnable
per-edge log-radius) through the C ABI against the oracle, on both pose-graph
solvers: iterates, objectives (1/2 sum rho(s)), implicit gradients including
the radius gradient, plus the adaptive / dogleg optimizers and the DLM
backward with Welsch edges.  Tolerances as for plain least squares: FP64
max(1e-10, 0.5 cond(H) eps64) per graph, mixed 1e-5."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import synth
from oracle import solve as S

from gpu_util import oracle_graphs, rel, t

pytestmark = pytest.mark.gpu
rng = np.random.default_rng(6060)


def _problem(seed, batch=4):
    p = synth.walk_se3(batch=batch, n_poses=16, n_loops=10, seed=seed, outliers=2)
    p["edge_logw"] = rng.normal(scale=0.2, size=len(p["edge_logw"]))
    p["edge_logc"] = rng.normal(np.log(0.5), 0.3, size=len(p["edge_logw"]))
    tau = 0.01 * rng.normal(size=(len(p["edge_logw"]), 6))
    return p, tau


def _run(p, tau, K, lam, solver="dense", precision="fp64", refine=0, adaptive=False, dogleg=None,
         mode="implicit", eps=1e-3):
    from paper_2207_09442_amd import Plan
    plan = Plan(p, K, lam=lam, solver=solver, precision=precision, refine=refine, device="cuda",
                adaptive=adaptive, dogleg=dogleg)
    poses = t(p["poses_init"])
    aux = (t(p["edge_meas"]), t(p["edge_logw"]), t(p["prior_meas"]), t(p["prior_logw"]))
    tau_d, logc = t(tau), t(p["edge_logc"])
    obj, st = plan.solve(poses, *aux, edge_tau=tau_d, edge_logc=logc)
    seed = rng.normal(size=(int(p["pose_off"][-1]), 6))
    out = plan.backward(poses, *aux, st, t(seed), edge_tau=tau_d, edge_logc=logc, mode=mode, eps=eps)
    torch.cuda.synchronize()
    return plan, poses.cpu().numpy(), obj.cpu().numpy(), st.cpu().numpy(), seed, \
        {k: v.cpu().numpy() for k, v in out.items()}


def _compare(p, tau, K, lam, tol, grad_tol=None, **kw):
    plan, got, obj, st, seed, gr = _run(p, tau, K, lam, **kw)
    B = len(p["pose_off"]) - 1
    gs = oracle_graphs(p, tau)
    worst = [0.0, 0.0, 0.0]
    for b in range(B):
        g = gs[b]
        r = S.solve_graph(g, K, lam, tau=g.tau, adaptive=kw.get("adaptive", False), dogleg_radius=kw.get("dogleg"))
        assert st[b] == r.status == S.OK
        lo, hi = int(p["pose_off"][b]), int(p["pose_off"][b + 1])
        e0, e1 = int(p["edge_off"][b]), int(p["edge_off"][b + 1])
        q0, q1 = int(p["prior_off"][b]), int(p["prior_off"][b + 1])
        ep = rel(got[lo:hi], g.G.to_storage(r.X).numpy())
        eo = rel(obj[b], np.asarray(r.objective))
        if kw.get("mode", "implicit") == "dlm":
            Xb = g.G.from_storage(torch.as_tensor(got[lo:hi]))
            at = S.GraphResult(X=Xb, pts=None, objective=[], status=S.OK, lin=S.linearize_pose_graph(g, Xb, tau=g.tau))
            ref = S.dlm_grad_graph(g, at, torch.as_tensor(seed[lo:hi]), kw["eps"])
        else:
            ref = S.implicit_grad_graph(g, r, torch.as_tensor(seed[lo:hi]))
        mine = np.concatenate([gr["edge_logw"][e0:e1], gr["edge_logc"][e0:e1], gr["edge_tau"][e0:e1].ravel(),
                               gr["prior_logw"][q0:q1]])
        theirs = np.concatenate([ref["edge_logw"].detach().numpy(), ref["edge_logc"].detach().numpy(),
                                 ref["tau"].detach().numpy().ravel(), ref["prior_logw"].detach().numpy()])
        eg = rel(mine, theirs)
        ev = np.linalg.eigvalsh(r.lin.H.numpy())
        gt = grad_tol if grad_tol is not None else max(tol, 0.5 * (ev[-1] / ev[0]) * np.finfo(np.float64).eps)
        worst = [max(worst[0], ep), max(worst[1], eo), max(worst[2], eg)]
        assert ep < tol and eo < tol * (1e3 if kw.get("precision") == "mixed" else 1) and eg < gt, (b, ep, eo, eg, gt)
    print(f"\n[welsch {kw}] pose {worst[0]:.2e} objective {worst[1]:.2e} grad {worst[2]:.2e}")


@pytest.mark.parametrize("solver", ["dense", "sparse"])
def test_welsch_fp64(solver):
    p, tau = _problem(61)
    _compare(p, tau, 8, 1e-3, 1e-10, solver=solver)


def test_welsch_mixed_refined():
    p, tau = _problem(62)
    _compare(p, tau, 8, 1e-3, 1e-5, grad_tol=1e-5, precision="mixed", refine=1)


@pytest.mark.parametrize("solver", ["dense", "sparse"])
def test_welsch_adaptive(solver):
    p, tau = _problem(63)
    _compare(p, tau, 6, 1e-2, 1e-10, solver=solver, adaptive=True)


def test_welsch_dogleg():
    p, tau = _problem(64)
    _compare(p, tau, 6, 0.0, 1e-10, dogleg=0.5)


@pytest.mark.parametrize("solver", ["dense", "sparse"])
def test_welsch_dlm(solver):
    p, tau = _problem(65)
    _compare(p, tau, 8, 1e-3, 1e-10, grad_tol=1e-8, solver=solver, mode="dlm", eps=1e-3)


def test_welsch_huge_radius_equals_least_squares_and_unsupported_modes():
    from paper_2207_09442_amd import DnlsError, Plan
    p, tau = _problem(66, batch=2)
    p["edge_logc"] = np.full(len(p["edge_logw"]), 30.0)
    _, a, oa, _, _, ga = _run(p, tau, 5, 1e-3)
    q = dict(p)
    plan = Plan(q, 5, lam=1e-3, device="cuda")
    poses = t(q["poses_init"])
    aux = (t(q["edge_meas"]), t(q["edge_logw"]), t(q["prior_meas"]), t(q["prior_logw"]))
    ob, st = plan.solve(poses, *aux, edge_tau=t(tau))
    assert rel(a, poses.cpu().numpy()) < 1e-12 and rel(oa, ob.cpu().numpy()) < 1e-12
    assert np.abs(ga["edge_logc"]).max() < 1e-12
    for mode in ("exact", "unroll"):
        with pytest.raises(DnlsError):
            plan.backward(poses, *aux, st, t(np.zeros((int(p["pose_off"][-1]), 6))), edge_tau=t(tau),
                          edge_logc=t(p["edge_logc"]), mode=mode)


def test_welsch_radius_through_the_autograd_layer():
    """The paper's PGO learning target: the loss sum ||X - X_gt||^2 on the
    3x4 storage, back-propagated by Layer / DNLSFunction into the Welsch
    log-radii (and log-weights), equals the oracle's implicit gradient with
    the seed taken by autograd through the retraction."""
    from paper_2207_09442_amd import Layer, Plan
    from oracle import lie
    p, tau = _problem(67, batch=2)
    K = 8
    plan = Plan(p, K, lam=1e-3, device="cuda")
    logc = t(p["edge_logc"]).requires_grad_(True)
    logw = t(p["edge_logw"]).requires_grad_(True)
    sol, info = Layer(plan).forward({"poses": t(p["poses_init"]), "edge_meas": t(p["edge_meas"]),
                                     "edge_logw": logw, "edge_tau": t(tau), "prior_meas": t(p["prior_meas"]),
                                     "edge_logc": logc})
    ((sol["poses"] - t(p["poses_gt"])) ** 2).sum().backward()
    assert info["status"].cpu().tolist() == [0, 0]
    gs = oracle_graphs(p, tau)
    ref_c, ref_w = [], []
    for b, g in enumerate(gs):
        r = S.solve_graph(g, K, 1e-3, tau=g.tau)
        lo, hi = p["pose_off"][b], p["pose_off"][b + 1]
        xi = torch.zeros(r.X.shape[0], 6, dtype=torch.float64, requires_grad=True)
        Y = lie.SE3.to_storage(lie.SE3.retract(r.X, xi))
        (v,) = torch.autograd.grad(((Y - torch.as_tensor(p["poses_gt"][lo:hi])) ** 2).sum(), [xi])
        o = S.implicit_grad_graph(g, r, v)
        ref_c.append(o["edge_logc"].detach().numpy())
        ref_w.append(o["edge_logw"].detach().numpy())
    assert rel(logc.grad.cpu().numpy(), np.concatenate(ref_c)) < 1e-8
    assert rel(logw.grad.cpu().numpy(), np.concatenate(ref_w)) < 1e-8
