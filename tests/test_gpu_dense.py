"""GPU parity of the pose-graph paths (C-ABI -> HIP kernels) against the CPU
oracle on the same seeded inputs.  The edge cases (SE(2), ragged batches with
weights and measurement tangents, mixed precision, K = 0, failed graphs, a
single-pose graph) run on both the dense and the block-sparse solver.

Tolerances
  FP64 path: 1e-10 relative per graph for poses, objective and gradients.
    The oracle's own spread under a permuted summation order is ~1e-15 on
    poses and ~1e-11 on gradients at condition numbers ~4e8, so 1e-10 leaves
    an order of magnitude for the different Cholesky blocking.  On the
    256-pose walks cond(H) reaches 1e11 and the oracle's gradient moves by
    up to 3e-10 under the same permutation (about 0.03 cond(H) eps); there the
    gradient is held to max(1e-10, 0.5 cond(H) eps), the forward-error bound
    of a backward-stable solve with a constant ten times the observed one.
  MIXED path (float32 linearisation and J^T J assembly, float64 factor):
    1e-5 relative for poses and gradients with one float64 refinement sweep;
    without refinement only the poses are held to 1e-5 (the gradient of these
    ill-conditioned graphs moves by ~1e-4, reported, not gated).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import solve as S

from gpu_util import (ew_ratio, gpu_backward, gpu_solve, oracle_grad_at, oracle_grad_spread, oracle_grads,
                      oracle_order_spread, oracle_solve, per_graph_rel, rel, stationary_equivalent, t)

pytestmark = pytest.mark.gpu
rng = np.random.default_rng(77)


def _seeds(p, poses_ref_by_graph, graphs):
    """Loss L = sum ||Log(X_gt^-1 X)||^2 and its tangent seed per graph."""
    seeds = []
    for b, X in zip(graphs, poses_ref_by_graph):
        lo, hi = int(p["pose_off"][b]), int(p["pose_off"][b + 1])
        _, v = S.pose_error_loss_and_seed(p["group"], X, p["poses_gt"][lo:hi])
        seeds.append(v)
    return seeds


def _compare(p, K, lam, precision="fp64", refine=0, tau=None, graphs=None, tol_pose=1e-10, tol_grad=1e-10,
             gate_grad=True, solver="dense", adaptive=False, dogleg=None, refine_last=0, pair=False,
             pose_norm=False, sparse_solve="auto"):
    """Element-wise comparison with the oracle on `graphs` (all by default):
    status; poses (storage entries, floor 1e-3 of the graph's largest);
    objective history (relative per entry); gradients per field (edge
    log-weights, tangents, prior log-weights) against the graph's largest
    gradient element.  Float64 gradients are held to max(tol_grad, 3 s_b),
    s_b the oracle's own spread on graph b (gpu_util.oracle_grad_spread),
    mixed gradients element by element with floor 1e-3.  pose_norm: the
    mixed-precision variants outside the 1e-5 contract (no refinement, or
    refinement in some steps only) are held on their poses to the per-graph
    relative norm ||x - x_ref|| / ||x_ref|| (the error metric of the
    precision study) and report the element-wise figures and the objectives.
    Float64 objectives that differ by more than the tolerance are held to
    three times the oracle's own drift under another elimination order
    (gpu_util.oracle_order_spread) at theta_0 and theta_K, and in between
    also to 0.5 cond(H*) eps64, the forward error a float64 step may carry;
    the scaled ratio enters `worst_obj`."""
    plan, poses, objective, status, dev = gpu_solve(p, K, lam, precision, refine, tau, solver=solver,
                                                    adaptive=adaptive, dogleg=dogleg, refine_last=refine_last, pair=pair,
                                                    sparse_solve=sparse_solve)
    B = len(p["pose_off"]) - 1
    graphs = list(range(B)) if graphs is None else graphs
    gs, res = oracle_solve(p, K, lam, tau=tau, graphs=graphs, adaptive=adaptive, dogleg=dogleg)
    got = poses.cpu().numpy()
    G = gs[0].G
    mixed = precision == "mixed"
    ref_poses = [G.to_storage(r.X).numpy() for r in res]
    st = status.cpu().numpy()
    obj = objective.cpu().numpy()
    worst_pose = worst_obj = worst_pose_norm = 0.0
    pose_rel = {}
    stationary = []
    for gi, b in enumerate(graphs):
        lo, hi = int(p["pose_off"][b]), int(p["pose_off"][b + 1])
        assert st[b] == res[gi].status, (b, st[b], res[gi].status)
        ep = ew_ratio(got[lo:hi], ref_poses[gi], 1e-3)
        if not mixed and not pose_norm and ep >= tol_pose and res[gi].status == S.OK \
                and not adaptive and dogleg is None:
            # converged ill-conditioned graph: theta_K is unique only up to the
            # rounding floor of the gradient; check that the GPU's iterate is as
            # stationary as the oracle's (and report the element-wise gap)
            ok, n_gpu, n_ref, ds = stationary_equivalent(gs[gi], res[gi], got[lo:hi])
            print(f"\n  graph {b}: poses {ep:.2e} apart; oracle gradient norm {n_gpu:.2e} at the GPU's "
                  f"theta_K, {n_ref:.2e} at its own; objectives {ds:.1e} apart")
            assert ok, (b, ep, n_gpu, n_ref, ds)
            stationary.append(b)
        else:
            worst_pose = max(worst_pose, ep)
        pose_rel[b] = rel(got[lo:hi], ref_poses[gi])
        worst_pose_norm = max(worst_pose_norm, pose_rel[b])
        ro = np.asarray(res[gi].objective)
        eo = ew_ratio(obj[b], ro, 1e-12)
        if not mixed and eo >= max(tol_pose, 1e-12) and res[gi].status == S.OK and not adaptive \
                and dogleg is None:
            # S at theta_0 and theta_K: held to three times the oracle's own
            # drift under another elimination order; the objectives after the
            # early steps also to 0.5 cond(H*) eps64, the forward error a
            # float64 step may carry on an ill-conditioned graph
            _, so = oracle_order_spread(gs[gi], K, lam)
            cond = float(np.linalg.cond(res[gi].lin.H.numpy()))
            tol_e = max(tol_pose, 3.0 * so)
            tol_i = max(tol_e, 0.5 * cond * 2.2e-16)
            ends = [0, K]
            ee = ew_ratio(obj[b][ends], ro[ends], 1e-12)
            ei = ew_ratio(obj[b][1:K], ro[1:K], 1e-12) if K > 1 else 0.0
            print(f"\n  graph {b}: objectives {ee:.2e} apart at theta_0 / theta_K, {ei:.2e} in between; the "
                  f"oracle's own drift {so:.2e}, cond(H*) {cond:.1e}: tolerances {tol_e:.1e} / {tol_i:.1e}")
            eo = max(ee / max(1.0, tol_e / max(tol_pose, 1e-12)), ei / max(1.0, tol_i / max(tol_pose, 1e-12)))
        worst_obj = max(worst_obj, eo)
    # backward with the seed of the oracle's solution (same v on both sides)
    seeds = _seeds(p, ref_poses, graphs)
    full_seed = np.zeros((p["pose_off"][-1], G.dof))
    for gi, b in enumerate(graphs):
        full_seed[p["pose_off"][b]:p["pose_off"][b + 1]] = seeds[gi]
    gr = gpu_backward(plan, poses, status, dev, full_seed, want_adjoint=True)
    ref = oracle_grads(gs, res, seeds)
    worst_grad = 0.0
    over = []
    for gi, b in enumerate(graphs):
        e0, e1 = int(p["edge_off"][b]), int(p["edge_off"][b + 1])
        q0, q1 = int(p["prior_off"][b]), int(p["prior_off"][b + 1])
        fields = [(gr["edge_logw"][e0:e1], ref[gi]["edge_logw"]), (gr["edge_tau"][e0:e1], ref[gi]["tau"]),
                  (gr["prior_logw"][q0:q1], ref[gi]["prior_logw"])]
        scale = max([float(np.abs(r).max()) for _, r in fields if np.size(r)] + [0.0])
        if scale == 0.0:
            err = max(float(np.abs(m).max()) if np.size(m) else 0.0 for m, _ in fields)
        else:
            err = max(ew_ratio(m, r, 1.0 if not mixed else 1e-3, scale) for m, r in fields)
        worst_grad = max(worst_grad, err)
        if err >= tol_grad:
            tol_b = tol_grad
            if not mixed and res[gi].status == S.OK:
                tol_b = max(tol_grad, 3.0 * oracle_grad_spread(gs[gi], res[gi], seeds[gi], pose_rel[b]))
                if err >= tol_b or b in stationary:
                    # the backward at a shared point: the oracle's gradient at the
                    # GPU's theta_K, so that only the backward's own rounding is
                    # compared (the forward's difference was checked above)
                    sh = oracle_grad_at(gs[gi], res[gi], got[int(p["pose_off"][b]):int(p["pose_off"][b + 1])],
                                        seeds[gi])
                    shf = [(m, r) for (m, _), r in zip(fields, [sh["edge_logw"], sh["tau"], sh["prior_logw"]])]
                    sscale = max([float(np.abs(r).max()) for _, r in shf if np.size(r)] + [0.0])
                    err_sh = max(ew_ratio(m, r, 1.0, sscale) for m, r in shf)
                    print(f"\n  graph {b}: gradient {err:.2e} from the oracle's, {err_sh:.2e} from the "
                          f"oracle's at the GPU's theta_K")
                    err = err_sh
            if err >= tol_b:
                over.append((b, err, tol_b))
    print(f"\n[{solver} {precision} refine={refine}] pose {worst_pose:.2e} (norm {worst_pose_norm:.2e}) "
          f"objective {worst_obj:.2e} grad {worst_grad:.2e}")
    assert (worst_pose_norm if pose_norm else worst_pose) < tol_pose
    if not pose_norm:
        assert worst_obj < (1e-5 if mixed else max(tol_pose, 1e-12))
    if gate_grad:
        assert not over, over
    if adaptive or dogleg is not None:
        # same accept / reject decisions: a rejected step repeats the objective exactly
        for gi, b in enumerate(graphs):
            rep_gpu = [obj[b][t + 1] == obj[b][t] for t in range(K)]
            rep_ref = [res[gi].objective[t + 1] == res[gi].objective[t] for t in range(K)]
            assert rep_gpu == rep_ref, (b, rep_gpu, rep_ref)
    return worst_pose, worst_grad


@pytest.mark.parametrize("solver", ["dense", "sparse"])
def test_se2_circle_fp64(solver):
    """16-pose SE(2) circle, batch 1, 10 Gauss-Newton steps (48x48 system)."""
    p = synth.circle_se2()
    _compare(p, 10, 0.0, solver=solver)


@pytest.mark.parametrize("solver", ["dense", "sparse"])
def test_se3_uneven_ragged_fp64_with_weights_and_tau(solver):
    """Uneven small graphs (ragged tiles: n = 6N not a multiple of 16), random
    log-weights, non-zero measurement perturbation tau, LM damping."""
    p = synth.uneven_walk_se3(batch=6, n_min=3, n_max=40, seed=3)
    p["edge_logw"] = rng.normal(scale=0.3, size=len(p["edge_logw"]))
    p["prior_logw"] = rng.normal(scale=0.3, size=len(p["prior_logw"]))
    tau = 0.01 * rng.normal(size=(len(p["edge_logw"]), 6))
    _compare(p, 6, 1e-3, tau=tau, solver=solver)


@pytest.mark.parametrize("solver", ["dense", "sparse"])
def test_se2_batch_gn_fp64(solver):
    p = synth.circle_se2(batch=5, n_poses=24, n_loops=10, seed=5)
    _compare(p, 8, 0.0, solver=solver)


@pytest.mark.parametrize("refine", [1, 2])
@pytest.mark.parametrize("solver", ["dense", "sparse"])
def test_se3_mixed_refined(refine, solver):
    p = synth.walk_se3(batch=4, n_poses=40, n_loops=40, seed=11)
    _compare(p, 10, 1e-3, precision="mixed", refine=refine, tol_pose=1e-5, tol_grad=1e-5, solver=solver)


@pytest.mark.parametrize("solver", ["dense", "sparse"])
def test_se3_mixed_unrefined_poses(solver):
    """Mixed precision without the float64 refinement sweep (the first rung
    of the precision study, not the 1e-5 path): the float32 steps move the
    iterates by ~2e-6 on the per-graph norm (element-wise up to ~6e-4 of the
    floor on the smallest storage entries) and the gradient by ~1e-4; poses
    are held to 1e-5 on the norm, the rest is reported."""
    p = synth.walk_se3(batch=4, n_poses=40, n_loops=40, seed=11)
    _compare(p, 10, 1e-3, precision="mixed", refine=0, tol_pose=1e-5, gate_grad=False, solver=solver,
             pose_norm=True)


@pytest.mark.parametrize("solver", ["dense", "sparse"])
def test_k_zero_final_linearisation_only(solver):
    p = synth.walk_se3(batch=3, n_poses=10, n_loops=6, seed=13)
    _compare(p, 0, 1e-3, solver=solver)


def test_walk64_b128_all_graphs_fp64_and_mixed():
    """The 128 x 64-pose LM workload at full size, the bench's launch (pair
    schedule): every graph is compared with the oracle element by element."""
    p = synth.walk_se3(batch=128)
    _compare(p, 10, 1e-3, pair=True)
    _compare(p, 10, 1e-3, precision="mixed", refine=1, tol_pose=1e-5, tol_grad=1e-5, pair=True)


@pytest.mark.parametrize("window", [1, -3])
@pytest.mark.parametrize("solver", ["dense", "sparse"])
def test_walk64_b128_mixed_refined_in_some_steps_only(solver, window):
    """refine_last: float32 steps with the float64 refinement sweep in the
    last step only (1) or the first three (-3).  The float32 steps move the
    trajectory by ~1e-6, which the ten LM steps do not wash out: poses stay
    within 1e-5 of the oracle (measured 4e-7 to 2e-6) but gradients move by
    ~1e-5 (measured 1.1e-5 to 1.3e-5 on the norm), against 2e-10 when every
    step is refined: the option does not meet the mixed path's 1e-5 on
    gradients, which are reported here, not gated; it trades that accuracy
    for 13-17% of solve time and is not the bench's configuration."""
    p = synth.walk_se3(batch=128)
    _compare(p, 10, 1e-3, precision="mixed", refine=1, refine_last=window, graphs=[0, 21, 37, 64, 81, 100, 127],
             tol_pose=1e-5, gate_grad=False, solver=solver, pose_norm=True)


@pytest.mark.parametrize("solver", ["dense", "sparse"])
def test_failed_graphs_are_frozen(solver):
    """Graph 1 has an isolated pose (no cost touches it) and lambda = 0, so its
    Hessian has an exactly zero diagonal block (NOT_PD); graph 2 has a NaN
    measurement (NONFINITE).  Both keep their initial poses, repeat their
    objective and get zero gradients; graph 0 is unaffected."""
    p = synth.walk_se3(batch=3, n_poses=8, n_loops=4, seed=17)
    last = int(p["pose_off"][1]) + 7
    keep = ~((p["edge_ij"][:, 0] == last) | (p["edge_ij"][:, 1] == last))
    counts = [int(keep[p["edge_off"][b]:p["edge_off"][b + 1]].sum()) for b in range(3)]
    p["edge_ij"], p["edge_meas"], p["edge_logw"] = p["edge_ij"][keep], p["edge_meas"][keep], p["edge_logw"][keep]
    p["edge_off"] = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    p["edge_meas"] = p["edge_meas"].copy()
    p["edge_meas"][p["edge_off"][2] + 1, 0, 3] = np.nan
    plan, poses, objective, status, dev = gpu_solve(p, 5, 0.0, solver=solver)
    st = status.cpu().numpy()
    assert st.tolist() == [0, 1, 2]
    got = poses.cpu().numpy()
    for b in (1, 2):
        lo, hi = p["pose_off"][b], p["pose_off"][b + 1]
        assert np.array_equal(got[lo:hi], p["poses_init"][lo:hi])
    ob = objective.cpu().numpy()
    assert np.all(ob[1] == ob[1][0])
    assert np.all(np.isnan(ob[2]))
    gs, res = oracle_solve(p, 5, 0.0, graphs=[0, 1])
    assert res[1].status == S.NOT_PD
    assert rel(got[: p["pose_off"][1]], gs[0].G.to_storage(res[0].X).numpy()) < 1e-10
    seed = rng.normal(size=(p["pose_off"][-1], 6))
    gr = gpu_backward(plan, poses, status, dev, seed)
    for b in (1, 2):
        e0, e1 = p["edge_off"][b], p["edge_off"][b + 1]
        assert np.all(gr["edge_logw"][e0:e1] == 0) and np.all(gr["edge_tau"][e0:e1] == 0)


@pytest.mark.parametrize("solver", ["dense", "sparse"])
def test_single_pose_graph_and_prior_only(solver):
    """Degenerate graph: one pose, no edges, only its prior (n = 6 -> padded 16)."""
    p = synth.walk_se3(batch=2, n_poses=2, n_loops=0, seed=19)
    # make graph 0 a single pose: keep pose 0 only
    q = {k: v for k, v in p.items()}
    q["pose_off"] = np.array([0, 1, 3], np.int32)
    q["poses_gt"] = np.concatenate([p["poses_gt"][:1], p["poses_gt"][2:]])
    q["poses_init"] = np.concatenate([p["poses_init"][:1], p["poses_init"][2:]])
    q["edge_off"] = np.array([0, 0, 1], np.int32)
    q["edge_ij"] = p["edge_ij"][1:] - 1
    q["edge_meas"] = p["edge_meas"][1:]
    q["edge_logw"] = p["edge_logw"][1:]
    q["prior_var"] = np.array([0, 1], np.int32)
    q["poses_init"][0, :, 3] += 0.3
    _compare(q, 3, 0.0, solver=solver)


def test_projection_operator_matches_tangent_gradient():
    """proj_X(dL/dX) equals d/dxi L(X Exp(xi)) at xi = 0 (Appendix D)."""
    from paper_2207_09442_amd import project_grad
    from oracle import lie
    for G, name in [(lie.SE3, "SE3"), (lie.SE2, "SE2")]:
        n = 37
        xi0 = torch.as_tensor(rng.normal(size=(n, G.dof)), dtype=torch.float64)
        X = G.exp(xi0)
        W = torch.as_tensor(rng.normal(size=G.to_storage(X).shape), dtype=torch.float64)
        Xs = G.to_storage(X).clone().requires_grad_(True)
        L = (W * Xs).sum() + (Xs ** 2).sum()
        (gX,) = torch.autograd.grad(L, [Xs])
        xi = torch.zeros(n, G.dof, dtype=torch.float64, requires_grad=True)
        L2 = (W * G.to_storage(G.retract(X, xi))).sum() + (G.to_storage(G.retract(X, xi)) ** 2).sum()
        (ref,) = torch.autograd.grad(L2, [xi])
        got = project_grad(name, t(G.to_storage(X).reshape(n, -1)), t(gX.reshape(n, -1))).cpu().numpy()
        assert rel(got, ref.numpy()) < 1e-12


def test_autograd_layer_end_to_end():
    """Layer.forward / loss.backward through the torch.autograd.Function."""
    from paper_2207_09442_amd import Layer, Plan
    from oracle import lie
    p = synth.walk_se3(batch=3, n_poses=12, n_loops=8, seed=23)
    plan = Plan(p, 6, lam=1e-3, device=t(0.0).device)
    logw = t(p["edge_logw"]).requires_grad_(True)
    tau = torch.zeros(len(p["edge_logw"]), 6, dtype=torch.float64, device=logw.device, requires_grad=True)
    sol, info = Layer(plan).forward({"poses": t(p["poses_init"]), "edge_meas": t(p["edge_meas"]),
                                     "edge_logw": logw, "edge_tau": tau, "prior_meas": t(p["prior_meas"])})
    X = sol["poses"]
    gt = t(p["poses_gt"])
    loss = ((X - gt) ** 2).sum()
    loss.backward()
    assert info["status"].cpu().numpy().tolist() == [0, 0, 0]
    # oracle: same loss on the 3x4 storage, seed by autograd through the retraction
    gs, res = oracle_solve(p, 6, 1e-3)
    seeds = []
    for g, r, b in zip(gs, res, range(3)):
        lo, hi = p["pose_off"][b], p["pose_off"][b + 1]
        xi = torch.zeros(r.X.shape[0], 6, dtype=torch.float64, requires_grad=True)
        Y = lie.SE3.to_storage(lie.SE3.retract(r.X, xi))
        Lb = ((Y - torch.as_tensor(p["poses_gt"][lo:hi])) ** 2).sum()
        (v,) = torch.autograd.grad(Lb, [xi])
        seeds.append(v.numpy())
    ref = oracle_grads(gs, res, seeds)
    ref_logw = np.concatenate([o["edge_logw"] for o in ref])
    ref_tau = np.concatenate([o["tau"] for o in ref])
    assert rel(logw.grad.cpu().numpy(), ref_logw) < 1e-9
    assert rel(tau.grad.cpu().numpy(), ref_tau) < 1e-9


def test_uneven_b256_sampled_graphs():
    """256 graphs with N uniform in [32, 256] in one launch (largest first),
    10 Gauss-Newton steps; the smallest, the largest and two other graphs
    are checked against the oracle in both precisions."""
    p = synth.uneven_walk_se3(batch=256)
    sizes = np.diff(p["pose_off"])
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 7, 200})
    _compare(p, 10, 0.0, graphs=pick)
    # cond(H) up to 1e11: three float64 refinement sweeps per step keep the
    # early Gauss-Newton objectives within 1e-5 (one sweep: 6e-4)
    _compare(p, 10, 0.0, precision="mixed", refine=3, graphs=pick, tol_pose=1e-5, tol_grad=1e-5)


@pytest.mark.parametrize("solver", ["dense", "sparse"])
def test_gpu_implicit_gradient_against_oracle_unrolled(solver):
    """The GPU implicit gradient against the oracle's unrolled gradient
    (autograd through the K Gauss-Newton steps): on a low-noise graph the two
    differ only by the residual-proportional Gauss-Newton term (the oracle
    pin measures 1.6e-4 at this noise level), while the GPU matches the
    oracle's own implicit gradient to 1e-10."""
    import dataclasses
    from oracle import lie
    p = synth.walk_se3(batch=1, n_poses=12, n_loops=6, sigma_t=0.0005, sigma_r=0.0001, seed=3)
    K = 25
    g = S.graphs_of(p)[0]
    logw = g.logw_e.clone().requires_grad_(True)
    tau = torch.zeros(g.ei.shape[0], 6, dtype=torch.float64, requires_grad=True)
    r = S.solve_graph(dataclasses.replace(g, logw_e=logw, tau=tau), K, 0.0)
    Xg = lie.SE3.from_storage(torch.as_tensor(p["poses_gt"]))
    L = (lie.SE3.log(lie.SE3.inv(Xg) @ r.X) ** 2).sum()
    gw, gt = torch.autograd.grad(L, [logw, tau])
    unrolled = np.concatenate([gw.numpy(), gt.numpy().ravel()])
    plan, poses, objective, status, dev = gpu_solve(p, K, 0.0, solver=solver)
    _, v = S.pose_error_loss_and_seed("SE3", poses.cpu().numpy(), p["poses_gt"])
    gr = gpu_backward(plan, poses, status, dev, v)
    mine = np.concatenate([gr["edge_logw"], gr["edge_tau"].ravel()])
    gap = rel(mine, unrolled)
    print(f"\n[{solver}] GPU implicit vs oracle unrolled: {gap:.2e}")
    assert gap < 1e-3



def _single_pose_rotation(group, theta0):
    from oracle import lie
    G = lie.group(group)
    d = G.dof
    P = G.exp(torch.as_tensor(np.array([[0.3, -0.2, 0.1, 0.05, -0.1, 0.2][:d]]), dtype=torch.float64))
    rot = np.zeros((1, d))
    rot[0, d - 1] = theta0
    X0 = P @ G.exp(torch.as_tensor(rot, dtype=torch.float64))
    st = lambda X: G.to_storage(X).numpy()
    return {"group": group, "pose_off": np.array([0, 1], np.int32), "poses_init": st(X0), "poses_gt": st(P),
            "edge_off": np.array([0, 0], np.int32), "edge_ij": np.zeros((0, 2), np.int32),
            "edge_meas": st(P)[:0], "edge_logw": np.zeros(0), "prior_off": np.array([0, 1], np.int32),
            "prior_var": np.array([0], np.int32), "prior_meas": st(P), "prior_logw": np.zeros(1)}


@pytest.mark.parametrize("solver", ["dense", "sparse"])
@pytest.mark.parametrize("group", ["SE2", "SE3"])
def test_adaptive_lm_closed_form_single_pose(group, solver):
    """Adaptive damping from lambda = 1 on a pure-rotation prior error:
    theta_K = theta_0 prod_t lambda_t / (1 + lambda_t), lambda_t = 10^-t.
    K = 3 keeps theta_K (3e-4) far from the rounding floor, where the loss
    seed and the prior-weight gradient (both O(theta^2)) are still
    meaningful."""
    from oracle import lie
    theta0, K = 0.7, 3
    p = _single_pose_rotation(group, theta0)
    plan, poses, objective, status, dev = gpu_solve(p, K, 1.0, adaptive=True, solver=solver)
    theta, lam = theta0, 1.0
    for _ in range(K):
        theta *= lam / (1.0 + lam)
        lam = max(lam / 10.0, 1e-7)
    G = lie.group(group)
    X = G.from_storage(torch.as_tensor(poses.cpu().numpy()))
    err = G.log(G.inv(G.from_storage(torch.as_tensor(p["prior_meas"]))) @ X)[0].numpy()
    expect = np.zeros(G.dof)
    expect[-1] = theta
    assert np.abs(err - expect).max() < 1e-12 * theta0
    _compare(p, K, 1.0, adaptive=True, solver=solver)


@pytest.mark.parametrize("solver", ["dense", "sparse"])
def test_adaptive_lm_rejects_and_recovers(solver):
    """SE(2) circle from a poor initial guess: the first two steps are
    rejected; the GPU takes the same decisions as the oracle and matches its
    poses, objectives and implicit gradients."""
    from oracle import lie
    p = synth.circle_se2(batch=1, seed=3)
    rng_ = np.random.default_rng(13)
    X = lie.SE2.from_storage(torch.as_tensor(p["poses_init"]))
    xi = torch.zeros(X.shape[0], 3, dtype=torch.float64)
    xi[:, 2] = torch.as_tensor(rng_.normal(scale=1.6, size=X.shape[0]))
    xi[:, :2] = torch.as_tensor(rng_.normal(scale=1.6, size=(X.shape[0], 2)))
    p["poses_init"] = lie.SE2.to_storage(lie.SE2.retract(X, xi)).numpy()
    _compare(p, 6, 1e-4, adaptive=True, solver=solver)


@pytest.mark.parametrize("solver", ["dense", "sparse"])
def test_adaptive_lm_se3_batch_fp64_and_mixed(solver):
    """Five adaptive steps from composed odometry stop far from convergence,
    so each step's residual error stays in theta_K: one float64 refinement
    sweep per step leaves gradients up to 4.6e-5 off element-wise, two
    sweeps are the mixed path's setting here (1e-5)."""
    p = synth.uneven_walk_se3(batch=6, n_min=16, n_max=60, seed=31)
    _compare(p, 5, 1e-2, adaptive=True, solver=solver)
    _compare(p, 5, 1e-2, precision="mixed", refine=2, tol_pose=1e-5, tol_grad=1e-5, adaptive=True, solver=solver)
    _compare(p, 5, 1e-2, precision="mixed", refine=0, tol_pose=1e-5, gate_grad=False, adaptive=True, solver=solver,
             pose_norm=True)


# ---------------------------------------------------------------------------
# Dogleg (trust region), dense and block-sparse solvers
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("solver", ["dense", "sparse"])
@pytest.mark.parametrize("group", ["SE2", "SE3"])
def test_dogleg_closed_form_single_pose(group, solver):
    """Pure-rotation prior error 1.0 with radius 0.1: the scaled-gradient
    steps leave 0.9, 0.7, 0.3 (the radius doubles on the boundary) and the
    Gauss-Newton step then lands on the target: objectives 0.5, 0.405, 0.245,
    0.045, 0."""
    from test_oracle_solve import _single_pose_rotation_problem
    p = _single_pose_rotation_problem(group, 1.0)
    plan, poses, objective, status, dev = gpu_solve(p, 4, 0.0, dogleg=0.1, solver=solver)
    assert status.cpu().tolist() == [0]
    ob = objective.cpu().numpy()[0]
    assert ob[:4] == pytest.approx([0.5, 0.405, 0.245, 0.045], rel=1e-12)
    assert abs(ob[4]) < 1e-24
    assert np.abs(poses.cpu().numpy()[0] - p["prior_meas"][0]).max() < 1e-12


@pytest.mark.parametrize("solver", ["dense", "sparse"])
@pytest.mark.parametrize("precision,refine,tol", [("fp64", 0, 1e-10), ("mixed", 1, 1e-5)])
def test_dogleg_se3_batch_with_rejections(precision, refine, tol, solver):
    """SE(3) batch from a very poor initial guess (rotations perturbed by
    2.5 rad): graph 2's first Gauss-Newton step raises the objective and is
    refused (radius 100 -> 17.7, then doubling), the others take full steps.
    Same iterates, objectives, accept/reject pattern and implicit gradients as
    the oracle; K = 6 stops well above the rounding floor, where accept/reject
    decisions would be decided by the last bit."""
    p = synth.walk_se3(batch=4, n_poses=10, n_loops=10, seed=48, init_noise=(3.0, 2.5))
    _compare(p, 6, 0.0, precision=precision, refine=refine, tol_pose=tol, tol_grad=tol, dogleg=100.0,
             solver=solver)


@pytest.mark.parametrize("solver", ["dense", "sparse"])
def test_dogleg_uneven_with_weights_tau_and_damping(solver):
    p = synth.uneven_walk_se3(batch=6, n_min=3, n_max=40, seed=23)
    p["edge_logw"] = rng.normal(scale=0.3, size=len(p["edge_logw"]))
    tau = 0.01 * rng.normal(size=(len(p["edge_logw"]), 6))
    _compare(p, 8, 1e-3, tau=tau, dogleg=0.05, solver=solver)


@pytest.mark.parametrize("schedule", ["sweeps", "workgroup"])
def test_dogleg_sparse_schedules_and_graph_replay(schedule):
    """The block-sparse dogleg under the per-column and one-workgroup
    schedules, and replayed from a captured HIP graph: every replay gives
    the eager result bit for bit."""
    from paper_2207_09442_amd import Plan
    p = synth.walk_se3(batch=3, n_poses=24, n_loops=12, seed=49, init_noise=(1.0, 0.8))
    plan = Plan(p, 6, lam=0.0, solver="sparse", device="cuda", dogleg=2.0, sparse_solve=schedule)
    gplan = Plan(p, 6, lam=0.0, solver="sparse", device="cuda", dogleg=2.0, sparse_solve=schedule, graph=True)
    aux = (t(p["edge_meas"]), t(p["edge_logw"]), t(p["prior_meas"]), t(p["prior_logw"]))
    x0 = t(p["poses_init"])
    ob0, st0 = plan.solve(x0, *aux)
    torch.cuda.synchronize()
    gs, res = oracle_solve(p, 6, 0.0, dogleg=2.0)
    for b, r in enumerate(res):
        lo, hi = int(p["pose_off"][b]), int(p["pose_off"][b + 1])
        assert int(st0[b]) == r.status == S.OK
        assert rel(x0.cpu().numpy()[lo:hi], gs[0].G.to_storage(r.X).numpy()) < 1e-10
        assert rel(ob0.cpu().numpy()[b], r.objective) < 1e-10
    for _ in range(3):
        x1 = t(p["poses_init"])
        ob1, st1 = gplan.solve(x1, *aux)
        torch.cuda.synchronize()
        assert torch.equal(x0, x1) and torch.equal(ob0, ob1) and torch.equal(st0, st1)


@pytest.mark.parametrize("mode,kw", [("dlm", {"eps": 1e-3}), ("exact", {"sweeps": 6}), ("unroll", {"steps": 3})])
def test_autograd_layer_backward_modes(mode, kw):
    """Layer(plan, backward_mode=...) runs the chosen backward through torch
    autograd: the gradients equal those of plan.backward with the same mode
    and the seed the layer builds (tangent projection of dLoss/dX)."""
    from paper_2207_09442_amd import Layer, Plan, project_grad
    p = synth.walk_se3(batch=2, n_poses=10, n_loops=6, seed=31)
    plan = Plan(p, 5, lam=1e-3, device=t(0.0).device, keep_iterates=(mode == "unroll"))
    logw = t(p["edge_logw"]).requires_grad_(True)
    tau = torch.zeros(len(p["edge_logw"]), 6, dtype=torch.float64, device=logw.device, requires_grad=True)
    sol, info = Layer(plan, backward_mode=mode, **kw).forward(
        {"poses": t(p["poses_init"]), "edge_meas": t(p["edge_meas"]), "edge_logw": logw, "edge_tau": tau,
         "prior_meas": t(p["prior_meas"])})
    X = sol["poses"]
    ((X - t(p["poses_gt"])) ** 2).sum().backward()
    seed = project_grad("SE3", X.detach().reshape(plan.V, -1), (2 * (X.detach() - t(p["poses_gt"]))).reshape(plan.V, -1))
    ref = plan.backward(X.detach(), t(p["edge_meas"]), t(p["edge_logw"]), t(p["prior_meas"]),
                        torch.zeros(plan.P, dtype=torch.float64, device=logw.device), info["status"], seed,
                        edge_tau=torch.zeros_like(tau), mode=mode, **kw)
    torch.cuda.synchronize()
    assert torch.equal(logw.grad, ref["edge_logw"]) and torch.equal(tau.grad, ref["edge_tau"])
