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
correct float64 implementations cannot be told apart on this graph.  Inputs come from the seeded generators in synth/;
everything else from oracle/.  About twelve minutes on one core:

    python tests/golden/make_sparse_goldens.py
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
    out = os.path.join(HERE, name + ".npz")
    np.savez_compressed(out, poses=poses, objective=np.asarray(res.objective), status=np.int32(res.status),
                        seed=v, edge_logw=gr["edge_logw"].detach().numpy(), tau=gr["tau"].detach().numpy(),
                        prior_logw=gr["prior_logw"].detach().numpy(), K=np.int32(c["K"]), lam=np.float64(c["lam"]),
                        graph=np.int32(b), grad_spread=np.float64(spread))
    print(f"{name}: {time.time() - t0:.0f} s, objective {res.objective[0]:.6e} -> {res.objective[-1]:.6e}, "
          f"gradient spread {spread:.2e}",
          flush=True)
    return out


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(CASES)):
        make(name)
