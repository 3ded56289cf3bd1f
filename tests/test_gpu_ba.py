"""GPU parity of the bundle-adjustment (Schur) path against the CPU oracle.

Element by element per problem: cameras (3x4 storage) and points with a
floor of 1e-3 of the problem's largest entry, objective histories relative
per entry, gradients per field (observation weights, prior log-weights,
per-observation Huber radii) against the problem's largest gradient element
(float64) or with a floor of 1e-3 of it (mixed).  FP64 path 1e-10; mixed
path (float32 Jacobians and assembly, float64 Schur complement and factor,
float64 final linearisation) 1e-5."""
import numpy as np
import pytest
import torch

import synth
from oracle import lie
from oracle import solve as S

from gpu_util import ew_ratio, rel, t

pytestmark = pytest.mark.gpu
rng = np.random.default_rng(5)


def _run(p, K, lam, precision="fp64", problems=None, tol=1e-10, seed_points=True, pair=False, adaptive=False,
         dogleg=None, solver="schur"):
    from paper_2207_09442_amd import Plan
    plan = Plan(p, K, lam=lam, solver=solver, precision=precision, device=t(0.0).device, pair=pair,
                adaptive=adaptive, dogleg=dogleg)
    assert plan.schedule()["pair"] == pair
    cams, pts = t(p["poses_init"]), t(p["points_init"])
    dev = dict(obs_uv=t(p["obs_uv"]), obs_w=t(p["obs_w"]), prior_meas=t(p["prior_meas"]),
               prior_logw=t(p["prior_logw"]))
    objective, status = plan.solve_ba(cams, pts, **dev)
    torch.cuda.synchronize()
    B = len(p["pose_off"]) - 1
    problems = list(range(B)) if problems is None else problems
    gs = S.graphs_of(p)
    st = status.cpu().numpy()
    got_c, got_p, obj = cams.cpu().numpy(), pts.cpu().numpy(), objective.cpu().numpy()
    seed_c = np.zeros((p["pose_off"][-1], 6))
    seed_p = np.zeros((p["point_off"][-1], 3))
    worst = dict(cam=0.0, pt=0.0, obj=0.0, grad=0.0)
    res = {}
    for b in problems:
        r = S.solve_graph(gs[b], K, lam, adaptive=adaptive, dogleg_radius=dogleg)
        res[b] = r
        assert st[b] == r.status
        c0, c1 = p["pose_off"][b], p["pose_off"][b + 1]
        q0, q1 = p["point_off"][b], p["point_off"][b + 1]
        worst["cam"] = max(worst["cam"], ew_ratio(got_c[c0:c1], lie.SE3.to_storage(r.X).numpy(), 1e-3))
        worst["pt"] = max(worst["pt"], ew_ratio(got_p[q0:q1], r.pts.numpy(), 1e-3))
        worst["obj"] = max(worst["obj"], ew_ratio(obj[b], np.asarray(r.objective), 1e-12))
        # seed: camera pose error (outer loss of the workload) plus a random point seed
        _, v = S.pose_error_loss_and_seed("SE3", lie.SE3.to_storage(r.X).numpy(), p["poses_gt"][c0:c1])
        seed_c[c0:c1] = v
        if seed_points:
            seed_p[q0:q1] = rng.normal(size=(q1 - q0, 3))
    gr = plan.backward_ba(cams, pts, status=status, seed_cam=t(seed_c), seed_pt=t(seed_p), **dev)
    torch.cuda.synchronize()
    gw, gl, gd = gr["obs_w"].cpu().numpy(), gr["prior_logw"].cpu().numpy(), gr["obs_delta"].cpu().numpy()
    for b in problems:
        c0, c1 = p["pose_off"][b], p["pose_off"][b + 1]
        q0, q1 = p["point_off"][b], p["point_off"][b + 1]
        o0, o1 = p["obs_off"][b], p["obs_off"][b + 1]
        r0, r1 = p["prior_off"][b], p["prior_off"][b + 1]
        ref = S.implicit_grad_graph(gs[b], res[b], torch.as_tensor(seed_c[c0:c1]), torch.as_tensor(seed_p[q0:q1]))
        fields = [(gw[o0:o1], ref["obs_w"].detach().numpy()), (gl[r0:r1], ref["prior_logw"].detach().numpy()),
                  (gd[o0:o1], ref["obs_delta"].detach().numpy())]
        scale = max(float(np.abs(r_).max()) for _, r_ in fields if np.size(r_))
        floor = 1e-3 if precision == "mixed" else 1.0
        worst["grad"] = max([worst["grad"]] + [ew_ratio(m, r_, floor, scale) for m, r_ in fields])
    print(f"\n[ba {precision}] " + " ".join(f"{k} {v:.2e}" for k, v in worst.items()))
    for k in ["cam", "pt", "grad", "obj"]:
        assert worst[k] < tol, (k, worst[k])
    return worst


@pytest.mark.parametrize("pair", [False, True])
def test_ba_small_fp64(pair):
    """pair: six workgroups per problem share the factorisation (one panel
    here, so most of them have no row group and only join the barrier)."""
    p = synth.bundle_adjustment(batch=2, n_cams=8, n_points=60, obs_per_point=4, seed=1)
    p["obs_w"] = np.exp(rng.normal(scale=0.2, size=len(p["obs_w"])))
    _run(p, 5, 1e-3, pair=pair)


def test_ba_uneven_problems_fp64():
    """Two problems of different camera counts (ragged camera systems, padding)."""
    a = synth.bundle_adjustment(batch=1, n_cams=9, n_points=50, obs_per_point=4, seed=2)
    b = synth.bundle_adjustment(batch=1, n_cams=14, n_points=70, obs_per_point=5, seed=3)
    p = {}
    for k in a:
        if k in ("group", "intrinsics", "huber_delta"):
            p[k] = a[k]
        elif k.endswith("_off"):
            p[k] = np.concatenate([a[k], a[k][-1] + b[k][1:]]).astype(np.int32)
        elif k in ("obs_cam", "prior_var"):
            p[k] = np.concatenate([a[k], b[k] + a["pose_off"][-1]]).astype(np.int32)
        elif k == "obs_pt":
            p[k] = np.concatenate([a[k], b[k] + a["point_off"][-1]]).astype(np.int32)
        else:
            p[k] = np.concatenate([a[k], b[k]])
    _run(p, 4, 1e-3)


@pytest.mark.parametrize("pair", [False, True])
def test_ba_ring64_full_size_fp64_and_mixed(pair):
    """4 problems x (64 cameras, 2048 points, 16384 observations), 10 LM
    steps, every problem compared; pair (the bench's launch): the 384 x 384
    camera systems factored by six workgroups each."""
    p = synth.bundle_adjustment(batch=4)
    _run(p, 10, 1e-3, pair=pair)
    _run(p, 10, 1e-3, precision="mixed", tol=1e-5, pair=pair)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_ba_sparse_elimination_small_and_ragged(precision, tol):
    """Bundle adjustment on the block-sparse solver (points eliminated first
    inside the tile factorisation, no explicit Schur complement): small and
    ragged problems with random observation weights against the oracle's
    Schur solution, cameras, points, objectives and gradients element by
    element, the implicit backward through the sparse factor."""
    from paper_2207_09442_amd import Plan
    p = synth.bundle_adjustment(batch=2, n_cams=8, n_points=60, obs_per_point=4, seed=1)
    p["obs_w"] = np.exp(rng.normal(scale=0.2, size=len(p["obs_w"])))
    assert Plan(p, 1, solver="sparse", device=t(0.0).device).schedule()["sparse_solve"] == "hybrid"
    _run(p, 5, 1e-3, precision=precision, tol=tol, solver="sparse")
    a = synth.bundle_adjustment(batch=1, n_cams=9, n_points=50, obs_per_point=4, seed=2)
    b = synth.bundle_adjustment(batch=1, n_cams=14, n_points=70, obs_per_point=5, seed=3)
    q = {}
    for k in a:
        if k in ("group", "intrinsics", "huber_delta"):
            q[k] = a[k]
        elif k.endswith("_off"):
            q[k] = np.concatenate([a[k], a[k][-1] + b[k][1:]]).astype(np.int32)
        elif k in ("obs_cam", "prior_var"):
            q[k] = np.concatenate([a[k], b[k] + a["pose_off"][-1]]).astype(np.int32)
        elif k == "obs_pt":
            q[k] = np.concatenate([a[k], b[k] + a["point_off"][-1]]).astype(np.int32)
        else:
            q[k] = np.concatenate([a[k], b[k]])
    _run(q, 4, 1e-3, precision=precision, tol=tol, solver="sparse")


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_ba_sparse_elimination_ring64_full_size(precision, tol):
    """The 4 x (64 cameras, 2048 points, 16384 observations) workload on the
    block-sparse solver (6528 unknowns per problem: the per-column solve
    sweeps), every problem against the oracle."""
    from paper_2207_09442_amd import Plan
    p = synth.bundle_adjustment(batch=4)
    assert Plan(p, 1, solver="sparse", device=t(0.0).device).schedule()["sparse_solve"] == "sweeps"
    _run(p, 10, 1e-3, precision=precision, tol=tol, solver="sparse")


def test_ba_sparse_elimination_refuses_other_modes():
    """The block-sparse BA path runs fixed damping and the implicit backward;
    adaptive damping, the dogleg and the DLM backward stay on the Schur
    solver."""
    from paper_2207_09442_amd import DnlsError, Plan
    p = synth.bundle_adjustment(batch=1, n_cams=8, n_points=40, obs_per_point=4, seed=5)
    for kw in (dict(adaptive=True), dict(dogleg=1.0), dict(sparse_solve="block")):
        with pytest.raises(DnlsError, match="not supported|takes the HYBRID|fixed-damping"):
            Plan(p, 3, lam=1e-3, solver="sparse", device=t(0.0).device, **kw)
    plan = Plan(p, 3, lam=1e-3, solver="sparse", device=t(0.0).device)
    cams, pts = t(p["poses_init"]), t(p["points_init"])
    dev = dict(obs_uv=t(p["obs_uv"]), obs_w=t(p["obs_w"]), prior_meas=t(p["prior_meas"]),
               prior_logw=t(p["prior_logw"]))
    _, status = plan.solve_ba(cams, pts, **dev)
    with pytest.raises(DnlsError, match="implicit backward only"):
        plan.backward_ba(cams, pts, status=status, seed_cam=torch.zeros(plan.V, 6, dtype=torch.float64,
                                                                        device=cams.device), mode="dlm", **dev)


@pytest.mark.parametrize("pair", [False, True])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_ba_adaptive_damping(precision, tol, pair):
    """Adaptive Levenberg-Marquardt on the Schur path: two problems from a
    fair start (every step kept, lambda / 10) and from a very poor one
    (cameras 1 rad / 3 m and points 2 off: steps 3 to 8 raise the objective
    and are refused, lambda x 10 each time, and the step at lambda = 0.1 is
    kept).  Same cameras, points, objectives (so the same accept / reject
    pattern) and gradients as the oracle."""
    _run(_fair_and_poor(), 10, 1e-7, precision=precision, tol=tol, pair=pair, adaptive=True)


def _fair_and_poor():
    """Two BA problems: the small ring from a fair start, and one from a very
    poor start (cameras 1 rad / 3 m and points 2 off)."""
    a = synth.bundle_adjustment(batch=1, n_cams=8, n_points=40, obs_per_point=4, seed=5)
    b = synth.bundle_adjustment(batch=1, n_cams=8, n_points=40, obs_per_point=4, cam_r=1.0, cam_t=3.0,
                                point_sigma=2.0, seed=2)
    p = {}
    for k in a:
        if k in ("group", "intrinsics", "huber_delta"):
            p[k] = a[k]
        elif k.endswith("_off"):
            p[k] = np.concatenate([a[k], a[k][-1] + b[k][1:]]).astype(np.int32)
        elif k in ("obs_cam", "prior_var"):
            p[k] = np.concatenate([a[k], b[k] + a["pose_off"][-1]]).astype(np.int32)
        elif k == "obs_pt":
            p[k] = np.concatenate([a[k], b[k] + a["point_off"][-1]]).astype(np.int32)
        else:
            p[k] = np.concatenate([a[k], b[k]])
    return p


@pytest.mark.parametrize("pair", [False, True])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
@pytest.mark.parametrize("radius", [1.0, 10.0])
def test_ba_dogleg(radius, precision, tol, pair):
    """Powell's dogleg over cameras and points on the Schur path: radius 1
    keeps the first steps on the boundary (doubling), radius 10 lets the
    poor start refuse its fourth step (radius 20 -> 4.67).  Same cameras,
    points, objectives and gradients as the oracle's full-system dogleg."""
    _run(_fair_and_poor(), 8, 0.0, precision=precision, tol=tol, pair=pair, dogleg=radius)


@pytest.mark.parametrize("pair", [False, True])
@pytest.mark.parametrize("eps", [1e-3, 0.3])
def test_ba_dlm_backward(eps, pair):
    """Direct loss minimisation on the Schur path against the oracle's
    full-system DLM at the cameras and points the GPU solve returned, with
    camera and point seeds; the factor cache afterwards serves the implicit
    backward exactly as before.  Tolerance: 1e-9 + 3e4 eps64 / eps + 0.5
    cond eps64 of the full system.  The eps-term is larger than for pose
    graphs: each camera's right-hand side sums hundreds of pixel-scale
    observation terms, whose rounding enters the step divided by eps (the
    GPU's Schur route and the oracle's full-system solve round differently);
    measured 1.9e-9 at eps = 1e-3 against 6.7e-9 from this term."""
    from paper_2207_09442_amd import Plan
    p = synth.bundle_adjustment(batch=2, n_cams=8, n_points=40, obs_per_point=4, seed=11)
    p["obs_w"] = np.exp(rng.normal(scale=0.2, size=len(p["obs_w"])))
    plan = Plan(p, 20, lam=1e-3, solver="schur", device=t(0.0).device, pair=pair)
    cams, pts = t(p["poses_init"]), t(p["points_init"])
    dev = dict(obs_uv=t(p["obs_uv"]), obs_w=t(p["obs_w"]), prior_meas=t(p["prior_meas"]),
               prior_logw=t(p["prior_logw"]))
    _, status = plan.solve_ba(cams, pts, **dev)
    vc = rng.normal(size=(int(p["pose_off"][-1]), 6))
    vp = rng.normal(size=(int(p["point_off"][-1]), 3))
    before = plan.backward_ba(cams, pts, status=status, seed_cam=t(vc), seed_pt=t(vp), want_adjoint=True, **dev)
    out = plan.backward_ba(cams, pts, status=status, seed_cam=t(vc), seed_pt=t(vp), mode="dlm", eps=eps, **dev)
    after = plan.backward_ba(cams, pts, status=status, seed_cam=t(vc), seed_pt=t(vp), want_adjoint=True, **dev)
    torch.cuda.synchronize()
    for k in before:
        assert rel(after[k].cpu().numpy(), before[k].cpu().numpy()) < 1e-13, k
    gw, gl, gd = out["obs_w"].cpu().numpy(), out["prior_logw"].cpu().numpy(), out["obs_delta"].cpu().numpy()
    st = status.cpu().numpy()
    gs = S.graphs_of(p)
    X_all, P_all = cams.cpu(), pts.cpu()
    e64 = np.finfo(np.float64).eps
    worst = 0.0
    for b in range(2):
        assert st[b] == S.OK
        g = gs[b]
        c0, c1 = p["pose_off"][b], p["pose_off"][b + 1]
        q0, q1 = p["point_off"][b], p["point_off"][b + 1]
        o0, o1 = p["obs_off"][b], p["obs_off"][b + 1]
        r0, r1 = p["prior_off"][b], p["prior_off"][b + 1]
        Xb, Pb = lie.SE3.from_storage(X_all[c0:c1]), P_all[q0:q1]
        res = S.GraphResult(X=Xb, pts=Pb, objective=[], status=S.OK, lin=S.linearize_ba(g, Xb, Pb))
        ref = S.dlm_grad_ba(g, res, vc[c0:c1], vp[q0:q1], eps)
        mine = np.concatenate([gw[o0:o1], gl[r0:r1], gd[o0:o1]])
        theirs = np.concatenate([ref["obs_w"].numpy(), ref["prior_logw"].numpy(), ref["obs_delta"].numpy()])
        ev = np.linalg.eigvalsh(S.ba_full_system(res.lin).numpy())
        tol = 1e-9 + 3e4 * e64 / eps + 0.5 * (ev[-1] / ev[0]) * e64
        err = rel(mine, theirs)
        worst = max(worst, err / tol)
        assert err < tol, (b, err, tol)
    print(f"\n[ba dlm eps={eps} pair={pair}] worst error / tolerance {worst:.2e}")


@pytest.mark.parametrize("dogleg", [None, 1.0])
def test_ba_failed_problem_is_frozen(dogleg):
    """Problem 1 loses every observation of one camera, whose block of the
    camera system is then singular at lambda = 0: the factorisation fails
    (NOT_PD), the problem keeps its cameras and points from that step on and
    repeats its objective, like the oracle's; problem 0 is untouched.  The
    implicit and DLM backward give problem 1 zero gradients."""
    from paper_2207_09442_amd import Plan
    p = _fair_and_poor()
    lost = int(p["pose_off"][1]) + 5
    keep = p["obs_cam"] != lost
    o1 = int(p["obs_off"][1])
    p["obs_off"] = np.array([0, int(keep[:o1].sum()), int(keep.sum())], np.int32)
    for k in ("obs_cam", "obs_pt", "obs_uv", "obs_w"):
        p[k] = p[k][keep]
    K = 4
    plan = Plan(p, K, lam=0.0, solver="schur", device=t(0.0).device, dogleg=dogleg)
    cams, pts = t(p["poses_init"]), t(p["points_init"])
    dev = dict(obs_uv=t(p["obs_uv"]), obs_w=t(p["obs_w"]), prior_meas=t(p["prior_meas"]),
               prior_logw=t(p["prior_logw"]))
    obj, status = plan.solve_ba(cams, pts, **dev)
    torch.cuda.synchronize()
    gs = S.graphs_of(p)
    res = [S.solve_graph(g, K, 0.0, dogleg_radius=dogleg) for g in gs]
    assert status.cpu().tolist() == [r.status for r in res] == [S.OK, S.NOT_PD]
    got_c, got_p, ob = cams.cpu().numpy(), pts.cpu().numpy(), obj.cpu().numpy()
    for b, r in enumerate(res):
        c0, c1 = p["pose_off"][b], p["pose_off"][b + 1]
        q0, q1 = p["point_off"][b], p["point_off"][b + 1]
        assert rel(got_c[c0:c1], lie.SE3.to_storage(r.X).numpy()) < 1e-10
        assert rel(got_p[q0:q1], r.pts.numpy()) < 1e-10
        assert rel(ob[b], np.asarray(r.objective)) < 1e-10
    vc = t(rng.normal(size=(int(p["pose_off"][-1]), 6)))
    o1 = int(p["obs_off"][1])
    for mode in ("implicit", "dlm"):
        gr = plan.backward_ba(cams, pts, status=status, seed_cam=vc, mode=mode, **dev)
        torch.cuda.synchronize()
        gw = gr["obs_w"].cpu().numpy()
        r1 = int(p["prior_off"][1])
        assert np.all(gw[o1:] == 0) and np.all(gr["prior_logw"].cpu().numpy()[r1:] == 0)
        assert np.all(gr["obs_delta"].cpu().numpy()[o1:] == 0)
        assert np.all(np.isfinite(gw[:o1])) and np.abs(gw[:o1]).max() > 0


def test_ba_autograd_layer_end_to_end():
    """BALayer.forward / loss.backward through DNLSFunctionBA: the gradients
    of a camera + point loss reach the observation weights and the prior
    log-weights, equal to the oracle's implicit gradient with the same seeds
    (camera seed by autograd through the retraction, point seed Euclidean)."""
    from paper_2207_09442_amd import BALayer, Plan
    p = synth.bundle_adjustment(batch=2, n_cams=8, n_points=40, obs_per_point=4, seed=13)
    p["obs_w"] = np.exp(rng.normal(scale=0.2, size=len(p["obs_w"])))
    plan = Plan(p, 6, lam=1e-3, solver="schur", device=t(0.0).device)
    obs_w = t(p["obs_w"]).requires_grad_(True)
    prior_logw = t(p["prior_logw"]).requires_grad_(True)
    sol, info = BALayer(plan).forward({"cams": t(p["poses_init"]), "points": t(p["points_init"]),
                                       "obs_uv": t(p["obs_uv"]), "obs_w": obs_w, "prior_meas": t(p["prior_meas"]),
                                       "prior_logw": prior_logw})
    loss = ((sol["cams"] - t(p["poses_gt"])) ** 2).sum() + ((sol["points"] - t(p["points_gt"])) ** 2).sum()
    loss.backward()
    assert info["status"].cpu().tolist() == [0, 0]
    gs = S.graphs_of(p)
    ref_w, ref_l = [], []
    for b, g in enumerate(gs):
        r = S.solve_graph(g, 6, 1e-3)
        c0, c1 = p["pose_off"][b], p["pose_off"][b + 1]
        q0, q1 = p["point_off"][b], p["point_off"][b + 1]
        xi = torch.zeros(r.X.shape[0], 6, dtype=torch.float64, requires_grad=True)
        Y = lie.SE3.to_storage(lie.SE3.retract(r.X, xi))
        (vc,) = torch.autograd.grad(((Y - torch.as_tensor(p["poses_gt"][c0:c1])) ** 2).sum(), [xi])
        vp = 2.0 * (r.pts - torch.as_tensor(p["points_gt"][q0:q1]))
        o = S.implicit_grad_graph(g, r, vc, vp)
        ref_w.append(o["obs_w"].detach().numpy())
        ref_l.append(o["prior_logw"].detach().numpy())
    assert rel(obs_w.grad.cpu().numpy(), np.concatenate(ref_w)) < 1e-9
    assert rel(prior_logw.grad.cpu().numpy(), np.concatenate(ref_l)) < 1e-9


def test_ba_autograd_layer_dlm_mode():
    """BALayer(plan, backward_mode="dlm") equals Plan.backward_ba in DLM mode
    with the seeds the layer builds."""
    from paper_2207_09442_amd import BALayer, Plan, project_grad
    p = synth.bundle_adjustment(batch=2, n_cams=8, n_points=40, obs_per_point=4, seed=14)
    plan = Plan(p, 6, lam=1e-3, solver="schur", device=t(0.0).device)
    obs_w = t(p["obs_w"]).requires_grad_(True)
    dev = dict(obs_uv=t(p["obs_uv"]), prior_meas=t(p["prior_meas"]), prior_logw=t(p["prior_logw"]))
    sol, info = BALayer(plan, backward_mode="dlm", eps=1e-2).forward(
        {"cams": t(p["poses_init"]), "points": t(p["points_init"]), "obs_w": obs_w, **dev})
    C, Q = sol["cams"], sol["points"]
    (((C - t(p["poses_gt"])) ** 2).sum() + ((Q - t(p["points_gt"])) ** 2).sum()).backward()
    seed_c = project_grad("SE3", C.detach().reshape(plan.V, -1), (2 * (C.detach() - t(p["poses_gt"]))).reshape(plan.V, -1))
    seed_p = 2 * (Q.detach() - t(p["points_gt"]))
    ref = plan.backward_ba(C.detach(), Q.detach(), obs_w=t(p["obs_w"]), status=info["status"], seed_cam=seed_c,
                           seed_pt=seed_p, mode="dlm", eps=1e-2, **dev)
    torch.cuda.synchronize()
    assert torch.equal(obs_w.grad, ref["obs_w"])


def test_ba_learnable_huber_radius_through_the_layer():
    """The robust kernel's radius as a per-problem solve input (the paper's
    BA example learns it): radii 1.5 and 3.0 px instead of the problem's 2;
    the solve equals the oracle's with those radii, and loss.backward gives
    the radius gradient (the sum of the per-observation ones) with the
    weight gradients, equal to the oracle's implicit gradient."""
    from paper_2207_09442_amd import BALayer, Plan
    p = synth.bundle_adjustment(batch=2, n_cams=8, n_points=40, obs_per_point=4, seed=15, pixel_sigma=2.0)
    plan = Plan(p, 6, lam=1e-3, solver="schur", device=t(0.0).device)
    radii = t([1.5, 3.0]).requires_grad_(True)
    obs_w = t(p["obs_w"]).requires_grad_(True)
    sol, info = BALayer(plan).forward({"cams": t(p["poses_init"]), "points": t(p["points_init"]),
                                       "obs_uv": t(p["obs_uv"]), "obs_w": obs_w, "prior_meas": t(p["prior_meas"]),
                                       "prior_logw": t(p["prior_logw"]), "huber_delta": radii})
    C, Q = sol["cams"], sol["points"]
    (((C - t(p["poses_gt"])) ** 2).sum() + ((Q - t(p["points_gt"])) ** 2).sum()).backward()
    assert info["status"].cpu().tolist() == [0, 0]
    gs = S.graphs_of(p)
    ref_d, ref_w = [], []
    for b, g in enumerate(gs):
        g.delta = [1.5, 3.0][b]
        r = S.solve_graph(g, 6, 1e-3)
        c0, c1 = p["pose_off"][b], p["pose_off"][b + 1]
        q0, q1 = p["point_off"][b], p["point_off"][b + 1]
        assert rel(C.detach().cpu().numpy()[c0:c1], lie.SE3.to_storage(r.X).numpy()) < 1e-10
        assert rel(Q.detach().cpu().numpy()[q0:q1], r.pts.numpy()) < 1e-10
        xi = torch.zeros(r.X.shape[0], 6, dtype=torch.float64, requires_grad=True)
        Y = lie.SE3.to_storage(lie.SE3.retract(r.X, xi))
        (vc,) = torch.autograd.grad(((Y - torch.as_tensor(p["poses_gt"][c0:c1])) ** 2).sum(), [xi])
        o = S.implicit_grad_graph(g, r, vc, 2.0 * (r.pts - torch.as_tensor(p["points_gt"][q0:q1])))
        lin = S.linearize_ba(g, r.X, r.pts)
        assert bool((lin.extra["drho"] < 1).any())          # some observations in the linear branch
        ref_d.append(float(o["obs_delta"].sum()))
        ref_w.append(o["obs_w"].detach().numpy())
    assert rel(radii.grad.cpu().numpy(), np.asarray(ref_d)) < 1e-9
    assert rel(obs_w.grad.cpu().numpy(), np.concatenate(ref_w)) < 1e-9


def test_ba_radius_checks_and_device_radius_gradient():
    """Per-problem Huber radii: a 0-dim radius is shared by every problem
    (same solve as the expanded [B] radius, gradient = the sum of the
    per-problem ones); float32, wrong shape and non-positive radii are
    refused; the per-problem radius gradient reduced by the library equals
    the per-problem sums of the per-observation ones."""
    from paper_2207_09442_amd import DnlsError, Plan
    p = synth.bundle_adjustment(batch=3, n_cams=8, n_points=40, obs_per_point=4, seed=16, pixel_sigma=2.0)
    plan = Plan(p, 5, lam=1e-3, solver="schur", device=t(0.0).device)
    dev = dict(obs_uv=t(p["obs_uv"]), obs_w=t(p["obs_w"]), prior_meas=t(p["prior_meas"]),
               prior_logw=t(p["prior_logw"]))
    runs = []
    for radii in (t(1.7), t([1.7, 1.7, 1.7])):
        cams, pts = t(p["poses_init"]), t(p["points_init"])
        obj, st = plan.solve_ba(cams, pts, huber_delta=radii, **dev)
        vc = t(np.random.default_rng(3).normal(size=(plan.V, 6)))
        gr = plan.backward_ba(cams, pts, status=st, seed_cam=vc, huber_delta=radii, **dev)
        torch.cuda.synchronize()
        runs.append((cams.cpu(), pts.cpu(), obj.cpu(), {k: v.cpu() for k, v in gr.items()}))
    assert torch.equal(runs[0][0], runs[1][0]) and torch.equal(runs[0][2], runs[1][2])
    gr = runs[1][3]
    off = p["obs_off"]
    sums = np.array([gr["obs_delta"].numpy()[off[b]:off[b + 1]].sum() for b in range(3)])
    assert np.abs(gr["huber_delta"].numpy() - sums).max() <= 1e-12 * np.abs(sums).max()
    assert np.abs(sums).max() > 0
    cams, pts = t(p["poses_init"]), t(p["points_init"])
    for bad in (torch.tensor([1.0, 2.0, 3.0], dtype=torch.float32, device=cams.device), t([1.0, 2.0]),
                t([1.0, 0.0, 2.0]), t([1.0, -1.0, 2.0])):
        with pytest.raises(DnlsError):
            plan.solve_ba(cams, pts, huber_delta=bad, **dev)
    # through the layer: a shared 0-dim radius gets the sum of the per-problem gradients
    from paper_2207_09442_amd import BALayer
    grads = []
    for radii in (t(1.7).requires_grad_(True), t([1.7, 1.7, 1.7]).requires_grad_(True)):
        sol, info = BALayer(plan).forward({"cams": t(p["poses_init"]), "points": t(p["points_init"]),
                                           "obs_w": t(p["obs_w"]), "huber_delta": radii, **dev})
        ((sol["cams"] - t(p["poses_gt"])) ** 2).sum().backward()
        grads.append(radii.grad.detach().cpu().numpy())
    assert grads[0].shape == () and grads[1].shape == (3,)
    assert abs(float(grads[0]) - grads[1].sum()) <= 1e-12 * np.abs(grads[1]).sum()


def test_backward_after_a_later_solve_is_refused():
    """The autograd functions save the plan's solve count: a second forward
    on the same Plan overwrites the factor cache, so backward of the first
    raises instead of using the other solve's factor."""
    from paper_2207_09442_amd import BALayer, DnlsError, Layer, Plan
    p = synth.bundle_adjustment(batch=1, n_cams=8, n_points=40, obs_per_point=4, seed=17)
    plan = Plan(p, 3, lam=1e-3, solver="schur", device=t(0.0).device)
    dev = dict(obs_uv=t(p["obs_uv"]), prior_meas=t(p["prior_meas"]), prior_logw=t(p["prior_logw"]))
    w1 = t(p["obs_w"]).requires_grad_(True)
    sol1, _ = BALayer(plan).forward({"cams": t(p["poses_init"]), "points": t(p["points_init"]), "obs_w": w1, **dev})
    sol2, _ = BALayer(plan).forward({"cams": t(p["poses_init"]), "points": t(p["points_init"]),
                                     "obs_w": t(p["obs_w"]).requires_grad_(True), **dev})
    with pytest.raises(DnlsError):
        (sol1["cams"] ** 2).sum().backward()
    (sol2["cams"] ** 2).sum().backward()            # the latest solve is fine
    q = synth.walk_se3(batch=2, n_poses=8, n_loops=4, seed=2)
    qplan = Plan(q, 3, lam=1e-3, device=t(0.0).device)
    inp = lambda: {"poses": t(q["poses_init"]), "edge_meas": t(q["edge_meas"]),
                   "edge_logw": t(q["edge_logw"]).requires_grad_(True), "prior_meas": t(q["prior_meas"])}
    s1, _ = Layer(qplan).forward(inp())
    Layer(qplan).forward(inp())
    with pytest.raises(DnlsError):
        (s1["poses"] ** 2).sum().backward()
