"""Shared helpers of the GPU parity tests: run the HIP path through the
C-ABI binding and the CPU oracle on the same seeded inputs."""
from __future__ import annotations

import numpy as np
import torch

from oracle import solve as S

DEV = torch.device("cuda:0") if torch.cuda.is_available() else None


def t(x, dtype=torch.float64):
    return torch.as_tensor(np.asarray(x), dtype=dtype, device=DEV).contiguous()


def rel(a, b):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def per_graph_rel(a, b, off):
    """max over graphs of ||a_b - b_b|| / ||b_b||"""
    worst = 0.0
    for g in range(len(off) - 1):
        lo, hi = int(off[g]), int(off[g + 1])
        if hi > lo:
            worst = max(worst, rel(a[lo:hi], b[lo:hi]))
    return worst


def ew_ratio(a, b, floor, scale=None):
    """Element-wise error ratio max_i |a_i - b_i| / max(|b_i|, floor * scale),
    scale = max |b| unless given (a graph's largest gradient element, say).
    A result within tol of the reference element by element has ratio <= tol."""
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    if b.size == 0:
        return 0.0
    s = float(np.abs(b).max()) if scale is None else float(scale)
    den = np.maximum(np.abs(b), floor * s)
    den = np.where(den > 0, den, 1.0)
    return float(np.max(np.abs(a - b) / den))


def oracle_grad_spread(g, res, v, pose_rel, seed=0):
    """How far the oracle's own implicit gradient (log-weights, tangents,
    prior log-weights) moves under rounding-level changes of its inputs:
    (i) the final linearisation summed in a permuted edge order, (ii) theta_K
    moved by a random right perturbation of relative size pose_rel (the
    measured pose difference between two float64 solves).  Returns the
    larger max-norm change relative to the gradient's max norm: the floor
    below which two correct float64 implementations cannot be told apart on
    this graph."""
    import dataclasses
    rng = np.random.default_rng(seed)
    vt = torch.as_tensor(np.asarray(v), dtype=torch.float64)
    G = g.G
    flat = lambda o, inv=None: np.concatenate([
        (o["edge_logw"].detach().numpy() if inv is None else o["edge_logw"].detach().numpy()[inv]),
        (o["tau"].detach().numpy() if inv is None else o["tau"].detach().numpy()[inv]).ravel(),
        o["prior_logw"].detach().numpy()])
    ref = flat(S.implicit_grad_graph(g, res, vt))
    scale = max(float(np.abs(ref).max()), 1e-300)
    perm = rng.permutation(len(g.ei))
    pt = torch.as_tensor(perm)
    gp = dataclasses.replace(g, ei=g.ei[pt], ej=g.ej[pt], Z=g.Z[pt], logw_e=g.logw_e[pt],
                             tau=None if g.tau is None else g.tau[pt],
                             logc_e=None if g.logc_e is None else g.logc_e[pt])
    lin = S.linearize_pose_graph(gp, res.X, tau=gp.tau)
    r1 = dataclasses.replace(res, lin=lin, factor=(torch.linalg.cholesky(lin.H),))
    a = flat(S.implicit_grad_graph(gp, r1, vt), inv=np.argsort(perm))
    st = G.to_storage(res.X)
    xi = torch.as_tensor(rng.normal(size=(res.X.shape[0], G.dof)), dtype=torch.float64)
    xi = xi / xi.norm() * max(pose_rel, 1e-14) * float(st.norm())
    X2 = G.retract(res.X, xi)
    lin2 = S.linearize_pose_graph(g, X2, tau=g.tau)
    r2 = dataclasses.replace(res, X=X2, lin=lin2, factor=(torch.linalg.cholesky(lin2.H),))
    b = flat(S.implicit_grad_graph(g, r2, vt))
    return max(np.abs(a - ref).max(), np.abs(b - ref).max()) / scale


def gpu_solve(p, K, lam, precision="fp64", refine=0, tau=None, solver="dense", adaptive=False, dogleg=None,
              refine_last=0, pair=False):
    from paper_2207_09442_amd import Plan
    plan = Plan(p, K, lam=lam, solver=solver, precision=precision, refine=refine, device=DEV, adaptive=adaptive,
                dogleg=dogleg, refine_last=refine_last, pair=pair)
    poses = t(p["poses_init"])
    dev = dict(edge_meas=t(p["edge_meas"]), edge_logw=t(p["edge_logw"]), prior_meas=t(p["prior_meas"]),
               prior_logw=t(p["prior_logw"]), edge_tau=None if tau is None else t(tau))
    objective, status = plan.solve(poses, dev["edge_meas"], dev["edge_logw"], dev["prior_meas"],
                                   dev["prior_logw"], edge_tau=dev["edge_tau"])
    torch.cuda.synchronize()
    return plan, poses, objective, status, dev


def gpu_backward(plan, poses, status, dev, seed, want_adjoint=False):
    out = plan.backward(poses, dev["edge_meas"], dev["edge_logw"], dev["prior_meas"], dev["prior_logw"],
                        status, t(seed), edge_tau=dev["edge_tau"], want_adjoint=want_adjoint)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def oracle_graphs(p, tau=None, graphs=None):
    gs = S.graphs_of(p)
    if tau is not None:
        for b, g in enumerate(gs):
            e0, e1 = int(p["edge_off"][b]), int(p["edge_off"][b + 1])
            g.tau = torch.as_tensor(np.asarray(tau[e0:e1]), dtype=torch.float64)
    if graphs is not None:
        gs = [gs[b] for b in graphs]
    return gs


def oracle_solve(p, K, lam, tau=None, graphs=None, adaptive=False, dogleg=None):
    """Oracle forward for all graphs (or the listed ones); returns
    (graphs, results)."""
    gs = oracle_graphs(p, tau, graphs)
    res = [S.solve_graph(g, K, lam, tau=g.tau, adaptive=adaptive, dogleg_radius=dogleg) for g in gs]
    return gs, res


def oracle_grads(gs, res, seeds):
    """seeds: list of [N_b, dof] arrays per graph."""
    out = []
    for g, r, v in zip(gs, res, seeds):
        o = S.implicit_grad_graph(g, r, torch.as_tensor(v, dtype=torch.float64))
        out.append({k: x.detach().numpy() for k, x in o.items()})
    return out
