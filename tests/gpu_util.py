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
              refine_last=0, pair=False, sparse_solve="auto"):
    from paper_2207_09442_amd import Plan
    if solver == "sparse-block":          # the block-sparse solver's BLOCK schedule
        solver, sparse_solve = "sparse", "block"
    plan = Plan(p, K, lam=lam, solver=solver, precision=precision, refine=refine, device=DEV, adaptive=adaptive,
                dogleg=dogleg, refine_last=refine_last, pair=pair, sparse_solve=sparse_solve)
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


def oracle_grad_at(g, res, poses_storage, v):
    """The oracle's implicit gradient (log-weights, tangents, prior
    log-weights, flattened) with the same seed v but at another theta_K, the
    GPU's: the final linearisation and its factor are recomputed there.  With
    it the backward is compared at a shared point, apart from the forward's
    own difference in theta_K."""
    import dataclasses
    G = g.G
    X = G.from_storage(torch.as_tensor(np.asarray(poses_storage), dtype=torch.float64))
    lin = S.linearize_pose_graph(g, X, tau=g.tau)
    r = dataclasses.replace(res, X=X, lin=lin, factor=(torch.linalg.cholesky(lin.H),))
    o = S.implicit_grad_graph(g, r, torch.as_tensor(np.asarray(v), dtype=torch.float64))
    return {k: x.detach().numpy() for k, x in o.items()}


def stationary_equivalent(g, res, poses_storage):
    """On a graph whose float64 iteration has converged to the rounding floor
    of its gradient, theta_K is fixed only up to that floor: along the soft
    modes of an ill-conditioned H many points have a gradient as small as the
    oracle's own, and two correct float64 implementations stop at different
    ones.  Returns (ok, gradient norm at the GPU's theta_K, at the oracle's,
    relative objective difference); ok when the oracle's converged gradient is
    below 1e-9 of its initial one, the GPU's theta_K has an oracle gradient
    at most twice the oracle's own and the objectives agree to 1e-12."""
    G = g.G
    X = G.from_storage(torch.as_tensor(np.asarray(poses_storage), dtype=torch.float64))
    g0 = float(S.linearize_pose_graph(g, g.X, tau=g.tau).g.norm())
    lin = S.linearize_pose_graph(g, X, tau=g.tau)
    n_gpu, n_ref = float(lin.g.norm()), float(res.lin.g.norm())
    ds = abs(float(lin.S) - float(res.lin.S)) / max(float(res.lin.S), 1e-300)
    ok = n_ref <= 1e-9 * g0 and n_gpu <= 2.0 * n_ref + 1e-15 * g0 and ds <= 1e-12
    return ok, n_gpu, n_ref, ds


def oracle_order_spread(g, K, lam):
    """How far the oracle's own K-step solve moves when every step solves its
    system in the reversed elimination order (the Cholesky factorisation of
    P (H + lambda I) P^T, P reversing the unknowns): the same steps in exact
    arithmetic, a different rounding of each factorisation.  Returns the
    element-wise differences (poses with a floor of 1e-3 of the largest
    entry, objective history per entry) from the oracle's result: on
    ill-conditioned graphs the early steps of two correct float64 solvers
    already differ by more than 1e-10 there."""
    G = g.G
    X = g.X.clone()
    obj = []
    for _ in range(K):
        lin = S.linearize_pose_graph(g, X, tau=g.tau)
        obj.append(float(lin.S))
        n = lin.H.shape[0]
        rev = torch.arange(n - 1, -1, -1)
        Lr = torch.linalg.cholesky(lin.H[rev][:, rev] + lam * torch.eye(n, dtype=torch.float64))
        d = torch.empty(n, dtype=torch.float64)
        d[rev] = torch.cholesky_solve(lin.g[rev][:, None], Lr)[:, 0]
        X = G.retract(X, -d.reshape(-1, G.dof))
    obj.append(float(S.linearize_pose_graph(g, X, tau=g.tau).S))
    ref = S.solve_graph(g, K, lam, tau=g.tau)
    return (ew_ratio(G.to_storage(X).numpy(), G.to_storage(ref.X).numpy(), 1e-3),
            ew_ratio(np.asarray(obj), np.asarray(ref.objective), 1e-12))
