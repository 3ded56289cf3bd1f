"""Writes the expected results of the full-size block-sparse parity tests:
the CPU oracle's sparse K-step solve (oracle.solve.solve_graph_sparse) and its
implicit gradient (Proposition 1) on

  lattice16_g0.npz  graph 0 of the 16^3 SE(3) lattice batch (4096 poses,
                    11520 lattice edges + 1152 long-range edges, prior on
                    pose 0), 15 Gauss-Newton steps;
  lattice11_sweeps.npz
                    the 11^3 lattice (1331 poses, seed 4), 4 Levenberg-
                    Marquardt steps at lambda = 1e-3, the graph that exceeds
                    the one-workgroup sparse solve.

The backward seed is the tangent gradient of L = sum_k ||Log(X_gt,k^-1 X_k)||^2
at the oracle's theta_K.  `grad_spread` is how far the oracle's own gradient
moves (max norm, relative to the gradient's max norm) when the final
linearisation is summed in a permuted edge order or theta_K is moved by a
random right perturbation of relative size 1e-13: the floor below which two
correct float64 implementations cannot be told apart on this graph.
`order_pose`, `order_objective` and `order_grad` are the element-wise
differences (poses with a floor of 1e-3 of the largest entry, objectives per
entry, gradients against the largest element) between this solve and the same
solve and backward on the graph with its poses relabelled at random, so that
minimum degree eliminates in another order: how far two correct float64
factorisations of these ill-conditioned systems drift apart through rounding
alone.  `cond` is cond(H*) at the stored theta_K (Lanczos), which bounds the
early objectives of a float64 solver: 0.5 cond(H*) eps64.  Inputs come from the seeded generators in synth/;
everything else from oracle/.  About twenty-five minutes on one core:

    python tests/golden/make_sparse_goldens.py            # everything
    python tests/golden/make_sparse_goldens.py --cond     # only the cond field
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth                                       # noqa: E402
from oracle import lie                             # noqa: E402
from oracle import solve as S                      # noqa: E402

CASES = {
    "lattice16_g0": dict(make=lambda: synth.lattice_se3(batch=8, side=16), graph=0, K=15, lam=0.0),
    "lattice11_sweeps": dict(make=lambda: synth.lattice_se3(batch=1, side=11, seed=4), graph=0, K=4, lam=1e-3),
}


def ew_ratio(a, b, floor):
    """max_i |a_i - b_i| / max(|b_i|, floor max |b|)"""
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    den = np.maximum(np.abs(b), floor * np.abs(b).max())
    return float(np.max(np.abs(a - b) / np.where(den > 0, den, 1.0)))


def relabelled(g, rng):
    """The graph with its poses renumbered by a random permutation (pose k of
    the new graph is pose perm[k] of the old one); edges and priors keep
    their order.  Returns (graph, perm)."""
    import dataclasses

    import torch
    perm = rng.permutation(g.X.shape[0])
    inv = torch.as_tensor(np.argsort(perm))
    return dataclasses.replace(g, X=g.X[torch.as_tensor(perm)], ei=inv[g.ei], ej=inv[g.ej], pv=inv[g.pv]), perm


def _flat(o, inv=None):
    e, t = o["edge_logw"].detach().numpy(), o["tau"].detach().numpy()
    if inv is not None:
        e, t = e[inv], t[inv]
    return np.concatenate([e, t.ravel(), o["prior_logw"].detach().numpy()])


def grad_spread(g, res, v, pose_rel=1e-13, seed=0) -> float:
    import dataclasses

    import torch
    rng = np.random.default_rng(seed)
    ref = _flat(S.implicit_grad_graph_sparse(g, res, v))
    scale = float(np.abs(ref).max())
    perm = rng.permutation(len(g.ei))
    pt = torch.as_tensor(perm)
    gp = dataclasses.replace(g, ei=g.ei[pt], ej=g.ej[pt], Z=g.Z[pt], logw_e=g.logw_e[pt])
    s, H, gv = S.linearize_pose_graph_sparse(gp, res.X)
    r1 = dataclasses.replace(res, factor=(S._sparse_factor(H),))
    a = _flat(S.implicit_grad_graph_sparse(gp, r1, v), inv=np.argsort(perm))
    st = lie.SE3.to_storage(res.X)
    xi = torch.as_tensor(rng.normal(size=(res.X.shape[0], 6)), dtype=torch.float64)
    X2 = lie.SE3.retract(res.X, xi / xi.norm() * pose_rel * float(st.norm()))
    s, H, gv = S.linearize_pose_graph_sparse(g, X2)
    r2 = dataclasses.replace(res, X=X2, factor=(S._sparse_factor(H),))
    b = _flat(S.implicit_grad_graph_sparse(g, r2, v))
    return max(np.abs(a - ref).max(), np.abs(b - ref).max()) / scale


def make(name: str) -> str:
    c = CASES[name]
    p = c["make"]()
    b = c["graph"]
    g = S.graphs_of(p)[b]
    t0 = time.time()
    res = S.solve_graph_sparse(g, c["K"], c["lam"])
    assert res.status == S.OK, res.status
    lo, hi = int(p["pose_off"][b]), int(p["pose_off"][b + 1])
    poses = lie.SE3.to_storage(res.X).numpy()
    _, v = S.pose_error_loss_and_seed("SE3", poses, p["poses_gt"][lo:hi])
    gr = S.implicit_grad_graph_sparse(g, res, v)
    spread = grad_spread(g, res, v)
    # the same solve and backward on the graph with its poses relabelled by a
    # random permutation: minimum degree then breaks its ties differently, so
    # every factorisation runs in another elimination order; the element-wise
    # drift between two correct float64 factorisations, per result
    g2, perm = relabelled(g, np.random.default_rng(7))
    alt = S.solve_graph_sparse(g2, c["K"], c["lam"])
    assert alt.status == S.OK, alt.status
    ga = S.implicit_grad_graph_sparse(g2, alt, v[perm])
    ref = _flat(gr)
    inv = np.argsort(perm)
    order_pose = ew_ratio(lie.SE3.to_storage(alt.X).numpy()[inv], poses, 1e-3)
    order_obj = ew_ratio(np.asarray(alt.objective), np.asarray(res.objective), 1e-12)
    order_grad = float(np.abs(_flat(ga) - ref).max() / np.abs(ref).max())
    out = os.path.join(HERE, name + ".npz")
    np.savez_compressed(out, poses=poses, objective=np.asarray(res.objective), status=np.int32(res.status),
                        seed=v, edge_logw=gr["edge_logw"].detach().numpy(), tau=gr["tau"].detach().numpy(),
                        prior_logw=gr["prior_logw"].detach().numpy(), K=np.int32(c["K"]), lam=np.float64(c["lam"]),
                        graph=np.int32(b), grad_spread=np.float64(spread), order_pose=np.float64(order_pose),
                        order_objective=np.float64(order_obj), order_grad=np.float64(order_grad))
    print(f"{name}: {time.time() - t0:.0f} s, objective {res.objective[0]:.6e} -> {res.objective[-1]:.6e}, "
          f"gradient spread {spread:.2e}; other elimination order: poses {order_pose:.2e}, "
          f"objective {order_obj:.2e}, gradient {order_grad:.2e}",
          flush=True)
    return out


def condition(name: str) -> float:
    """cond(H*) of the stored result (the oracle's final linearisation at its
    theta_K): largest eigenvalue by Lanczos, smallest by shift-invert Lanczos
    through the oracle's sparse factor.  Stored as `cond`: the condition-scaled
    bound 0.5 cond(H*) eps64 holds the early objectives of the float64 path."""
    import scipy.sparse.linalg as sla
    import torch
    c = CASES[name]
    p = c["make"]()
    g = S.graphs_of(p)[c["graph"]]
    path = os.path.join(HERE, name + ".npz")
    gd = dict(np.load(path))
    X = lie.SE3.from_storage(torch.as_tensor(gd["poses"]))
    _, H, _ = S.linearize_pose_graph_sparse(g, X)
    lmax = sla.eigsh(H, k=1, which="LA", return_eigenvectors=False)[0]
    lu = S._sparse_factor(H)
    op = sla.LinearOperator(H.shape, matvec=lambda x: lu.solve(np.asarray(x, dtype=np.float64).ravel()))
    mu = sla.eigsh(op, k=1, which="LA", return_eigenvectors=False)[0]   # 1 / smallest eigenvalue
    cond = float(lmax * mu)
    gd["cond"] = np.float64(cond)
    np.savez_compressed(path, **gd)
    print(f"{name}: cond(H*) {cond:.3e}", flush=True)
    return cond


if __name__ == "__main__":
    args = sys.argv[1:]
    if args and args[0] == "--cond":
        for name in (args[1:] or list(CASES)):
            condition(name)
    else:
        for name in (args or list(CASES)):
            make(name)
            condition(name)
