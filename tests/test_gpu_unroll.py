"""GPU parity of the unrolled and truncated backward (differentiation
through the optimizer's last steps) through the C ABI against the oracle's
unrolled_grad_graph (torch.autograd through the same steps).

The GPU recomputes each step in float64 at the iterates the solve kept and
runs the reverse sweep by hand (retraction adjoint, one solve with the step
matrix, the per-cost gradient of y^T g - y^T H delta); FP64 parity is held
to max(1e-10, 0.5 cond(H) eps64) per graph like the implicit gradient.  The
adjoint output dL/dtheta_{K-steps} is compared relative to the larger of its
own norm and the seed's (it vanishes once the steps have converged).
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import synth
from oracle import solve as S

from gpu_util import gpu_solve, oracle_graphs, rel, t

pytestmark = pytest.mark.gpu
rng = np.random.default_rng(5150)


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


def _unroll(p, tau, K, lam, steps=None, precision="fp64", refine=0, graphs=None, tol_floor=1e-10, solver="dense"):
    from paper_2207_09442_amd import Plan
    kw = dict(solver="sparse", sparse_solve="block") if solver == "sparse-block" else dict(solver=solver)
    plan = Plan(p, K, lam=lam, precision=precision, refine=refine, device="cuda", keep_iterates=True, **kw)
    poses = t(p["poses_init"])
    dev = dict(edge_meas=t(p["edge_meas"]), edge_logw=t(p["edge_logw"]), prior_meas=t(p["prior_meas"]),
               prior_logw=t(p["prior_logw"]), edge_tau=None if tau is None else t(tau))
    _, status = plan.solve(poses, dev["edge_meas"], dev["edge_logw"], dev["prior_meas"], dev["prior_logw"],
                           edge_tau=dev["edge_tau"])
    seed = rng.normal(size=(int(p["pose_off"][-1]), plan.dof))
    out = plan.backward(poses, dev["edge_meas"], dev["edge_logw"], dev["prior_meas"], dev["prior_logw"], status,
                        t(seed), edge_tau=dev["edge_tau"], want_adjoint=True, mode="unroll", steps=steps)
    torch.cuda.synchronize()
    gr = {k: v.cpu().numpy() for k, v in out.items()}
    st = status.cpu().numpy()
    B = len(p["pose_off"]) - 1
    graphs = list(range(B)) if graphs is None else graphs
    gs = oracle_graphs(p, tau, graphs)
    worst = 0.0
    for gi, b in enumerate(graphs):
        assert st[b] == S.OK
        g = gs[gi]
        lo, hi = int(p["pose_off"][b]), int(p["pose_off"][b + 1])
        ref = S.unrolled_grad_graph(g, K, lam, torch.as_tensor(seed[lo:hi]), steps=steps)
        e0, e1 = int(p["edge_off"][b]), int(p["edge_off"][b + 1])
        q0, q1 = int(p["prior_off"][b]), int(p["prior_off"][b + 1])
        mine = np.concatenate([gr["edge_logw"][e0:e1], gr["edge_tau"][e0:e1].ravel(), gr["prior_logw"][q0:q1]])
        theirs = np.concatenate([ref["edge_logw"].numpy(), ref["tau"].numpy().ravel(), ref["prior_logw"].numpy()])
        H = S.linearize_pose_graph(g, S.solve_graph(g, K, lam).X, tau=g.tau).H.numpy()
        ev = np.linalg.eigvalsh(H)
        tol = max(tol_floor, 0.5 * (ev[-1] / ev[0]) * np.finfo(np.float64).eps)
        # the adjoint dL/dtheta_{K-steps} vanishes where the steps have converged (theta_K then no
        # longer depends on the start): its error is measured against the seed's scale as well
        ra = ref["adjoint"].numpy()
        eg = rel(mine, theirs)
        ea = np.linalg.norm(gr["adjoint"][lo:hi] - ra) / max(np.linalg.norm(ra), np.linalg.norm(seed[lo:hi]))
        print(f"\n  graph {b}: gradient {eg:.2e} adjoint {ea:.2e} tolerance {tol:.2e}")
        worst = max(worst, eg / tol, ea / tol)
        assert eg < tol and ea < tol, (b, eg, ea, tol)
    return worst


@pytest.mark.parametrize("solver", ["dense", "sparse", "sparse-block"])
@pytest.mark.parametrize("group", ["SE2", "SE3"])
def test_unrolled_matches_oracle_ragged_batch(group, solver):
    p, tau = _problem(group, seed=51)
    _unroll(p, tau, 5, 1e-3, solver=solver)


@pytest.mark.parametrize("solver", ["dense", "sparse"])
@pytest.mark.parametrize("steps", [1, 3])
def test_truncated_matches_oracle(steps, solver):
    p, tau = _problem("SE3", seed=52)
    _unroll(p, tau, 6, 1e-2, steps=steps, solver=solver)


@pytest.mark.parametrize("solver", ["dense", "sparse"])
def test_unrolled_after_mixed_precision_solve(solver):
    """The reverse sweep runs in float64 at the iterates the mixed solve kept;
    those differ from the oracle's float64 iterates by ~1e-9 (refine = 1)."""
    p, tau = _problem("SE3", seed=53)
    _unroll(p, tau, 5, 1e-3, precision="mixed", refine=1, tol_floor=1e-5, solver=solver)


def test_unrolled_sparse_leaves_the_factor_cache_of_h_star():
    """The block-sparse reverse sweep factors each step's system in the factor
    cache and re-factors H* at the end: the implicit backward afterwards is
    bit-identical to the one before."""
    from paper_2207_09442_amd import Plan
    p, tau = _problem("SE3", seed=54)
    plan = Plan(p, 5, lam=1e-3, solver="sparse", device="cuda", keep_iterates=True)
    poses = t(p["poses_init"])
    aux = (t(p["edge_meas"]), t(p["edge_logw"]), t(p["prior_meas"]), t(p["prior_logw"]))
    _, status = plan.solve(poses, *aux, edge_tau=t(tau))
    seed = t(rng.normal(size=(int(p["pose_off"][-1]), 6)))
    before = plan.backward(poses, *aux, status, seed, edge_tau=t(tau), want_adjoint=True)
    plan.backward(poses, *aux, status, seed, edge_tau=t(tau), mode="unroll", steps=3)
    after = plan.backward(poses, *aux, status, seed, edge_tau=t(tau), want_adjoint=True)
    torch.cuda.synchronize()
    for k in before:
        assert torch.equal(before[k], after[k]), k


def test_unrolled_walk64_b128_sampled_graphs():
    p = synth.walk_se3(batch=128)
    _unroll(p, None, 10, 1e-3, graphs=[0, 81])


@pytest.mark.parametrize("solver", ["dense", "sparse"])
def test_unrolled_argument_checks_and_failed_graph(solver):
    from paper_2207_09442_amd import DnlsError, Plan
    p = synth.walk_se3(batch=2, n_poses=8, n_loops=4, seed=17)
    q = synth.bundle_adjustment(batch=1, n_cams=8, n_points=40, obs_per_point=4, seed=9)
    with pytest.raises(DnlsError):
        Plan(q, 4, solver="schur", device="cuda", keep_iterates=True)
    with pytest.raises(DnlsError):
        Plan(p, 4, lam=1e-3, device="cuda", keep_iterates=True, adaptive=True)
    last = int(p["pose_off"][1]) + 7
    keep = ~((p["edge_ij"][:, 0] == last) | (p["edge_ij"][:, 1] == last))
    counts = [int(keep[p["edge_off"][b]:p["edge_off"][b + 1]].sum()) for b in range(2)]
    p["edge_ij"], p["edge_meas"], p["edge_logw"] = p["edge_ij"][keep], p["edge_meas"][keep], p["edge_logw"][keep]
    p["edge_off"] = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    plan = Plan(p, 4, lam=0.0, device="cuda", keep_iterates=True, solver=solver)
    poses = t(p["poses_init"])
    aux = (t(p["edge_meas"]), t(p["edge_logw"]), t(p["prior_meas"]), t(p["prior_logw"]))
    _, status = plan.solve(poses, *aux)
    assert status.cpu().tolist() == [S.OK, S.NOT_PD]
    seed = t(rng.normal(size=(int(p["pose_off"][-1]), 6)))
    out = plan.backward(poses, *aux, status, seed, want_adjoint=True, mode="unroll")
    torch.cuda.synchronize()
    e0, lo = int(p["edge_off"][1]), int(p["pose_off"][1])
    assert torch.all(out["edge_logw"][e0:] == 0) and torch.all(out["adjoint"][lo:] == 0)
    assert torch.isfinite(out["edge_logw"][:e0]).all() and out["edge_logw"][:e0].abs().max() > 0
    for steps in (0, 5):
        with pytest.raises(DnlsError):
            plan.backward(poses, *aux, status, seed, mode="unroll", steps=steps)
    plain = Plan(p, 4, lam=0.0, device="cuda", solver=solver)
    plain.solve(poses.clone(), *aux)
    with pytest.raises(DnlsError):
        plain.backward(poses, *aux, status, seed, mode="unroll")
