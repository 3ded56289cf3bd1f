"""GPU parity of the block-sparse path (tile-supernodal Cholesky) against the
CPU oracle.  Small lattices and uneven walks are compared element by element
with the dense oracle (FP64 1e-10, mixed 1e-5).  The full-size lattices are
compared element by element with the sparse oracle's results written by
tests/golden/make_sparse_goldens.py (graph 0 of the 16^3 batch after 15
Gauss-Newton steps, the 11^3 graph of the per-column schedule after 4
damped steps), and through properties that hold at any size: the first
Gauss-Newton step solves (H + lambda I) delta = g to a small residual, and the
objective values at the initial and final iterates equal the oracle's
objective at those iterates."""
import os

import numpy as np
import pytest
import torch

import synth
from oracle import lie
from oracle import solve as S

from gpu_util import ew_ratio, gpu_backward, oracle_grads, oracle_solve, rel, t

pytestmark = pytest.mark.gpu


def _solve(p, K, lam, precision="fp64", refine=0):
    from paper_2207_09442_amd import Plan
    plan = Plan(p, K, lam=lam, solver="sparse", precision=precision, refine=refine, device=t(0.0).device)
    poses = t(p["poses_init"])
    dev = dict(edge_meas=t(p["edge_meas"]), edge_logw=t(p["edge_logw"]), prior_meas=t(p["prior_meas"]),
               prior_logw=t(p["prior_logw"]), edge_tau=None)
    objective, status = plan.solve(poses, dev["edge_meas"], dev["edge_logw"], dev["prior_meas"], dev["prior_logw"])
    torch.cuda.synchronize()
    return plan, poses, objective, status, dev


def _parity(p, K, lam, precision="fp64", refine=0, tol=1e-10, graphs=None, sparse_solve="auto", tau=None):
    """Element-wise comparison with the oracle on `graphs` (all by default),
    the dense tests' comparison on the block-sparse solver."""
    from test_gpu_dense import _compare
    return _compare(p, K, lam, precision=precision, refine=refine, graphs=graphs, tol_pose=tol, tol_grad=tol,
                    solver="sparse", sparse_solve=sparse_solve, tau=tau)


def test_lattice4_fp64():
    _parity(synth.lattice_se3(batch=2, side=4, seed=1), 5, 0.0)


def test_lattice6_fp64_and_mixed():
    p = synth.lattice_se3(batch=2, side=6, seed=2)
    _parity(p, 6, 0.0)
    _parity(p, 6, 0.0, precision="mixed", refine=1, tol=1e-5)


def test_uneven_walks_sparse_fp64():
    """Different structures per graph and n not a multiple of the tile size."""
    _parity(synth.uneven_walk_se3(batch=4, n_min=20, n_max=70, seed=9), 6, 1e-3)


@pytest.mark.parametrize("group", ["SE2", "SE3"])
def test_block_schedule_ragged(group):
    """The BLOCK schedule (pose-block factor, elimination-tree levels, one
    persistent launch) on ragged batches with weights, measurement tangents
    and damping, both precisions, against the oracle element by element."""
    if group == "SE3":
        p = synth.uneven_walk_se3(batch=6, n_min=3, n_max=60, seed=41)
    else:
        p = synth.circle_se2(batch=5, n_poses=30, n_loops=12, seed=42)
    rng = np.random.default_rng(43)
    p["edge_logw"] = rng.normal(scale=0.3, size=len(p["edge_logw"]))
    dof = 6 if group == "SE3" else 3
    tau = 0.01 * rng.normal(size=(len(p["edge_logw"]), dof))
    _parity(p, 6, 1e-3, sparse_solve="block", tau=tau)
    _parity(p, 6, 1e-3, precision="mixed", refine=1, tol=1e-5, sparse_solve="block", tau=tau)


def test_block_schedule_uneven_b256_sampled_graphs():
    """The 256-walk workload on the BLOCK schedule: the smallest, the largest
    and two other graphs against the oracle in both precisions."""
    p = synth.uneven_walk_se3(batch=256)
    sizes = np.diff(p["pose_off"])
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 7, 200})
    _parity(p, 10, 0.0, graphs=pick, sparse_solve="block")
    _parity(p, 10, 0.0, precision="mixed", refine=3, tol=1e-5, graphs=pick, sparse_solve="block")


def test_uneven_b256_full_size_sampled_graphs():
    """The 256-walk workload (N uniform in [32, 256]) on the sparse solver,
    10 Gauss-Newton steps in one batch; the smallest, the largest and two
    other graphs are compared with the oracle in both precisions."""
    p = synth.uneven_walk_se3(batch=256)
    sizes = np.diff(p["pose_off"])
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 7, 200})
    _parity(p, 10, 0.0, graphs=pick)
    # cond(H) up to 1e11: three float64 refinement sweeps per step keep the
    # early Gauss-Newton objectives within 1e-5 (one sweep: 6e-4)
    _parity(p, 10, 0.0, precision="mixed", refine=3, tol=1e-5, graphs=pick)


def test_lattice16_b8_full_size_properties():
    p = synth.lattice_se3(batch=8, side=16)
    # one step: delta solves (H + lambda I) delta = g at theta_0
    plan, poses, objective, status, dev = _solve(p, 1, 0.0)
    assert status.cpu().numpy().tolist() == [0] * 8
    got = poses.cpu().numpy()
    G = lie.SE3
    for b in (0, 5):
        lo, hi = p["pose_off"][b], p["pose_off"][b + 1]
        g = S.graphs_of(p)[b]
        s0, H, gv = S.linearize_pose_graph_sparse(g, g.X)
        X1 = G.from_storage(torch.as_tensor(got[lo:hi]))
        delta = -G.log(G.inv(g.X) @ X1).reshape(-1).numpy()
        r = H @ delta - gv
        print(f"\n[lattice16 graph {b}] step residual {np.linalg.norm(r) / np.linalg.norm(gv):.2e}")
        assert np.linalg.norm(r) < 1e-8 * np.linalg.norm(gv)
        assert abs(objective[b, 0].item() - s0) < 1e-10 * s0
        s1, _, _ = S.linearize_pose_graph_sparse(g, X1)
        assert abs(objective[b, 1].item() - s1) < 1e-10 * s1
    # the full 15-step solve in mixed precision: objective decreases, status ok
    plan, poses, objective, status, dev = _solve(p, 15, 0.0, precision="mixed", refine=1)
    ob = objective.cpu().numpy()
    assert status.cpu().numpy().tolist() == [0] * 8
    assert np.all(ob[:, -1] < ob[:, 0])


def test_sweep_solve_elementwise():
    """A batch whose largest graph exceeds the one-workgroup solve (more than
    6144 unknowns), so every graph is solved by the per-column / per-row
    sweeps: the small graphs are compared with the oracle element by element,
    the large one through the one-step residual."""
    big = synth.lattice_se3(batch=1, side=11, seed=4)          # 1331 poses, 7986 unknowns
    small = synth.uneven_walk_se3(batch=3, n_min=20, n_max=60, seed=5)
    p = {}
    for k in small:
        if k == "group":
            p[k] = small[k]
        elif k.endswith("_off"):
            p[k] = np.concatenate([small[k], small[k][-1] + big[k][1:]]).astype(np.int32)
        elif k in ("edge_ij", "prior_var"):
            p[k] = np.concatenate([small[k], big[k] + small["pose_off"][-1]]).astype(np.int32)
        else:
            p[k] = np.concatenate([small[k], big[k]])
    _parity(p, 4, 1e-3, graphs=[0, 1, 2])
    _parity(p, 4, 1e-3, precision="mixed", refine=1, tol=1e-5, graphs=[0, 1, 2])
    plan, poses, objective, status, dev = _solve(p, 1, 0.0)
    assert status.cpu().numpy().tolist() == [0, 0, 0, 0]
    b = 3
    lo, hi = p["pose_off"][b], p["pose_off"][b + 1]
    g = S.graphs_of(p)[b]
    _, H, gv = S.linearize_pose_graph_sparse(g, g.X)
    X1 = lie.SE3.from_storage(torch.as_tensor(poses.cpu().numpy()[lo:hi]))
    delta = -lie.SE3.log(lie.SE3.inv(g.X) @ X1).reshape(-1).numpy()
    r = H @ delta - gv
    print(f"\n[sweeps big graph] step residual {np.linalg.norm(r) / np.linalg.norm(gv):.2e}")
    assert np.linalg.norm(r) < 1e-8 * np.linalg.norm(gv)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden_parity(p, name, precision, refine, tol):
    """Solve the whole batch on the GPU, run the implicit backward with the
    golden seed on the golden's graph (zero seeds elsewhere) and compare that
    graph element by element with the stored oracle results: poses (floor
    1e-3 of the largest entry), objectives, gradients per field (float64:
    against the graph's largest gradient element, at max(tol, 3 s), s the
    oracle's own spread stored with the results; mixed: floor 1e-3).
    Float64 results are held to max(tol, 3 d), d the element-wise drift of
    the oracle's own result when its factorisations take another elimination
    order (stored with the results); the objectives after the early steps
    (t = 1 .. K-1) also to 0.5 cond(H*) eps64, the forward error a float64
    step may carry on these ill-conditioned systems (cond(H*) stored with the
    results), while theta_K, S_K and the gradient keep the tight bounds."""
    gd = np.load(os.path.join(GOLDEN, name + ".npz"))
    K, lam, b = int(gd["K"]), float(gd["lam"]), int(gd["graph"])
    plan, poses, objective, status, dev = _solve(p, K, lam, precision, refine)
    assert int(status[b]) == int(gd["status"]) == S.OK
    lo, hi = int(p["pose_off"][b]), int(p["pose_off"][b + 1])
    e0, e1 = int(p["edge_off"][b]), int(p["edge_off"][b + 1])
    q0, q1 = int(p["prior_off"][b]), int(p["prior_off"][b + 1])
    ep = ew_ratio(poses.cpu().numpy()[lo:hi], gd["poses"].reshape(hi - lo, -1), 1e-3)
    ob = objective.cpu().numpy()[b]
    ends = [0, K]                                   # S at theta_0 and at theta_K
    eo = ew_ratio(ob[ends], gd["objective"][ends], 1e-12)
    # the objectives after the early steps: a float64 solver's step carries
    # a forward error up to ~cond(H) eps64, so they are held to the
    # condition-scaled bound as well
    ei = ew_ratio(ob[1:K], gd["objective"][1:K], 1e-12) if K > 1 else 0.0
    seed = np.zeros((int(p["pose_off"][-1]), 6))
    seed[lo:hi] = gd["seed"]
    gr = gpu_backward(plan, poses, status, dev, seed)
    fields = [(gr["edge_logw"][e0:e1], gd["edge_logw"]), (gr["edge_tau"][e0:e1], gd["tau"]),
              (gr["prior_logw"][q0:q1], gd["prior_logw"])]
    scale = max(float(np.abs(r).max()) for _, r in fields)
    mixed = precision == "mixed"
    eg = max(ew_ratio(m, r, 1e-3 if mixed else 1.0, scale) for m, r in fields)
    tol_p = tol if mixed else max(tol, 3.0 * float(gd["order_pose"]))
    tol_o = tol if mixed else max(tol, 3.0 * float(gd["order_objective"]))
    tol_i = tol if mixed else max(tol_o, 0.5 * float(gd["cond"]) * 2.2e-16)
    tol_g = tol if mixed else max(tol, 3.0 * float(gd["grad_spread"]), 3.0 * float(gd["order_grad"]))
    print(f"\n[{name} {precision}] pose {ep:.2e} objective {eo:.2e} (intermediate {ei:.2e}) grad {eg:.2e} "
          f"(tolerances {tol_p:.1e} {tol_o:.1e} {tol_i:.1e} {tol_g:.1e})")
    assert ep < tol_p and eo < tol_o and ei < tol_i and eg < tol_g


@pytest.mark.parametrize("precision,refine,tol", [("fp64", 0, 1e-10), ("mixed", 2, 1e-5)])
def test_lattice16_b8_graph0_against_sparse_oracle(precision, refine, tol):
    """The 16^3 lattice workload at full size (8 graphs of 4096 poses, 15
    Gauss-Newton steps, the bench's launch); graph 0 against the sparse
    oracle, element by element.  Mixed precision takes two float64
    refinement sweeps per step here: with one, the objective after the first
    (large) Gauss-Newton step is 2.6e-5 off (cond(H) ~ 7e8), with two 4e-7."""
    _golden_parity(synth.lattice_se3(batch=8, side=16), "lattice16_g0", precision, refine, tol)


@pytest.mark.parametrize("precision,refine,tol", [("fp64", 0, 1e-10), ("mixed", 1, 1e-5)])
def test_lattice11_sweeps_against_sparse_oracle(precision, refine, tol):
    """The 11^3 lattice (7986 unknowns: beyond the one-workgroup sparse
    solve, so the per-column / per-row sweeps run) against the sparse
    oracle, element by element."""
    from paper_2207_09442_amd import Plan
    p = synth.lattice_se3(batch=1, side=11, seed=4)
    assert Plan(p, 1, solver="sparse", device=t(0.0).device).schedule()["sparse_solve"] == "sweeps"
    _golden_parity(p, "lattice11_sweeps", precision, refine, tol)
