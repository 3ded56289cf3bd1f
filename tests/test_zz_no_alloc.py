"""dnls_solve_noalloc (the solve with its workspace in the library's own
device array, for callers that cannot allocate) against dnls_solve on the
same inputs: two calls in a row, the second on a smaller problem, each
compared bit for bit (same kernels, same inputs), then the implicit backward
from each call's factor cache; and the argument checks."""
import ctypes

import numpy as np
import pytest
import torch

import synth

from gpu_util import t

pytestmark = pytest.mark.gpu


def _pose_inputs(p):
    return dict(edge_meas=t(p["edge_meas"]), edge_logw=t(p["edge_logw"]), prior_meas=t(p["prior_meas"]),
                prior_logw=t(p["prior_logw"]))


def _solve_pair(p, K, lam, **plan_kw):
    """The same problem through dnls_solve and dnls_solve_noalloc (separate
    plans, so each has its own factor cache); returns both runs."""
    from paper_2207_09442_amd import Plan
    runs = []
    for noalloc in (False, True):
        plan = Plan(p, K, lam=lam, device=t(0.0).device, **plan_kw)
        poses = t(p["poses_init"])
        dev = _pose_inputs(p)
        objective, status = plan.solve(poses, **dev, noalloc=noalloc)
        torch.cuda.synchronize()
        seed = torch.ones(plan.V, plan.dof, dtype=torch.float64, device=poses.device)
        g = plan.backward(poses, dev["edge_meas"], dev["edge_logw"], dev["prior_meas"], dev["prior_logw"], status,
                          seed)
        torch.cuda.synchronize()
        runs.append(dict(poses=poses.cpu().numpy(), objective=objective.cpu().numpy(),
                         status=status.cpu().numpy(), **{k: v.cpu().numpy() for k, v in g.items()}))
        plan.close()
    return runs


def _same(a, b, what):
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), (what, k, np.nanmax(np.abs(a[k] - b[k])))


def test_noalloc_matches_dnls_solve_two_calls_second_smaller():
    """First call: the 128 x 64-pose LM workload, mixed precision, pair
    schedule (the bench's launch); second call: a smaller ragged SE(3)
    batch in float64 on the dense solver.  The second call reuses the
    scratch the first one left behind."""
    print("\n[noalloc] walk64 b128 mixed pair", flush=True)
    big = synth.walk_se3(batch=128)
    a, b = _solve_pair(big, 10, 1e-3, precision="mixed", refine=1, pair=True)
    _same(a, b, "walk64_b128")
    print("[noalloc] uneven walks b6 fp64", flush=True)
    small = synth.uneven_walk_se3(batch=6, n_min=3, n_max=40, seed=3)
    a, b = _solve_pair(small, 6, 1e-3)
    _same(a, b, "uneven_b6")


def test_noalloc_sparse_and_schur_after_the_dense_call():
    """The other two solvers through the same scratch: a 4^3 lattice on the
    block-sparse solver, then a small bundle-adjustment batch."""
    from paper_2207_09442_amd import Plan
    print("\n[noalloc] lattice 4^3 sparse", flush=True)
    lat = synth.lattice_se3(batch=2, side=4, seed=2)
    a, b = _solve_pair(lat, 5, 0.0, solver="sparse")
    _same(a, b, "lattice4")
    print("[noalloc] bundle adjustment b2", flush=True)
    p = synth.bundle_adjustment(batch=2, n_cams=8, n_points=60, obs_per_point=4, seed=1)
    runs = []
    for noalloc in (False, True):
        plan = Plan(p, 5, lam=1e-3, solver="schur", device=t(0.0).device)
        cams, pts = t(p["poses_init"]), t(p["points_init"])
        dev = dict(obs_uv=t(p["obs_uv"]), obs_w=t(p["obs_w"]), prior_meas=t(p["prior_meas"]),
                   prior_logw=t(p["prior_logw"]))
        objective, status = plan.solve_ba(cams, pts, **dev, noalloc=noalloc)
        torch.cuda.synchronize()
        g = plan.backward_ba(cams, pts, status=status,
                             seed_cam=torch.ones(plan.V, 6, dtype=torch.float64, device=cams.device), **dev)
        torch.cuda.synchronize()
        runs.append(dict(cams=cams.cpu().numpy(), pts=pts.cpu().numpy(), objective=objective.cpu().numpy(),
                         status=status.cpu().numpy(), **{k: v.cpu().numpy() for k, v in g.items()}))
        plan.close()
    _same(runs[0], runs[1], "ba_b2")


def test_noalloc_argument_checks():
    """A workspace pointer, a HIP-graph plan and a plan whose solve workspace
    exceeds the scratch are refused before anything is enqueued."""
    import paper_2207_09442_amd as P
    from paper_2207_09442_amd import DnlsError, Plan
    p = synth.walk_se3(batch=2, n_poses=8, n_loops=4, seed=1)
    plan = Plan(p, 2, lam=1e-3, device=t(0.0).device)
    a = P._SolveArgs()
    poses = t(p["poses_init"])
    dev = _pose_inputs(p)
    obj = torch.empty(2, 3, dtype=torch.float64, device=poses.device)
    st = torch.empty(2, dtype=torch.int32, device=poses.device)
    a.poses, a.objective, a.status = P._ptr(poses), P._ptr(obj), P._ptr(st)
    a.edge_meas, a.edge_logw = P._ptr(dev["edge_meas"]), P._ptr(dev["edge_logw"])
    a.prior_meas, a.prior_logw = P._ptr(dev["prior_meas"]), P._ptr(dev["prior_logw"])
    a.factor = plan._aligned(plan.factor)
    a.workspace = plan._aligned(plan.workspace)
    code = P.lib().dnls_solve_noalloc(plan._h, ctypes.byref(a), P._stream())
    assert code == 1 and b"workspace must be NULL" in P.lib().dnls_last_error()
    plan.close()
    lat = synth.lattice_se3(batch=1, side=4)
    plan = Plan(lat, 2, solver="sparse", graph=True, device=t(0.0).device)
    with pytest.raises(DnlsError, match="DNLS_FLAG_GRAPH"):
        plan.solve(t(lat["poses_init"]), **_pose_inputs(lat), noalloc=True)
    plan.close()
    # 256 walks of up to 256 poses: the dense systems alone take ~2.4 GB of workspace
    big = synth.uneven_walk_se3(batch=256)
    plan = Plan(big, 1, device=t(0.0).device)
    assert plan.solve_ws_bytes > 256 << 20
    with pytest.raises(DnlsError, match="exceeds the scratch"):
        plan.solve(t(big["poses_init"]), **_pose_inputs(big), noalloc=True)
    plan.close()
