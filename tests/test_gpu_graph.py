"""Captured launch sequences (DNLS_FLAG_GRAPH) and forced sparse solve
schedules give the same results as the eager launches.  Every replay is
checked against the eager result, with eager work and host synchronisation
between the replays; a change of the argument pointers forces a new capture."""
import numpy as np
import pytest
import torch

import synth

from gpu_util import t

pytestmark = pytest.mark.gpu


def _pose_graph_run(p, plan, poses0):
    poses = poses0.clone()
    dev = [t(p["edge_meas"]), t(p["edge_logw"]), t(p["prior_meas"]), t(p["prior_logw"])]
    obj, st = plan.solve(poses, *dev)
    torch.cuda.synchronize()
    return poses.cpu().numpy(), obj.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("precision,refine", [("fp64", 0), ("mixed", 1)])
def test_sparse_graph_replays_match_eager(precision, refine):
    from paper_2207_09442_amd import Plan
    p = synth.uneven_walk_se3(batch=6, n_min=20, n_max=90, seed=21)
    poses0 = t(p["poses_init"])
    eager = Plan(p, 6, lam=1e-3, solver="sparse", precision=precision, refine=refine, device=poses0.device)
    ref = _pose_graph_run(p, eager, poses0)
    graph = Plan(p, 6, lam=1e-3, solver="sparse", precision=precision, refine=refine, device=poses0.device,
                 graph=True)
    poses = poses0.clone()
    dev = [t(p["edge_meas"]), t(p["edge_logw"]), t(p["prior_meas"]), t(p["prior_logw"])]
    for rep in range(4):
        poses.copy_(poses0)                       # eager work between replays
        obj, st = graph.solve(poses, *dev)        # same pointers: capture once, then replay
        torch.cuda.synchronize()
        assert np.array_equal(poses.cpu().numpy(), ref[0]), rep
        assert np.array_equal(obj.cpu().numpy(), ref[1]), rep
        assert np.array_equal(st.cpu().numpy(), ref[2]), rep
        _pose_graph_run(p, eager, poses0)         # other work on the stream
    # new pointers: recaptured
    got = _pose_graph_run(p, graph, poses0)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


@pytest.mark.parametrize("opt", [{}, {"adaptive": True}, {"dogleg": 1.0}])
def test_ba_graph_replays_match_eager(opt):
    """Fixed damping, adaptive damping and the dogleg on the Schur path (their
    decisions are taken on the device): every replay of the captured solve
    equals the eager one bit for bit."""
    from paper_2207_09442_amd import Plan
    p = synth.bundle_adjustment(batch=2, n_cams=10, n_points=80, obs_per_point=5, seed=3)
    dev = dict(obs_uv=t(p["obs_uv"]), obs_w=t(p["obs_w"]), prior_meas=t(p["prior_meas"]),
               prior_logw=t(p["prior_logw"]))
    c0, q0 = t(p["poses_init"]), t(p["points_init"])
    eager = Plan(p, 5, lam=1e-3, solver="schur", precision="mixed", device=c0.device, **opt)
    cams, pts = c0.clone(), q0.clone()
    obj_e, st_e = eager.solve_ba(cams, pts, **dev)
    torch.cuda.synchronize()
    ref = (cams.cpu().numpy(), pts.cpu().numpy(), obj_e.cpu().numpy())
    graph = Plan(p, 5, lam=1e-3, solver="schur", precision="mixed", device=c0.device, graph=True, **opt)
    cams, pts = c0.clone(), q0.clone()
    for rep in range(3):
        cams.copy_(c0)
        pts.copy_(q0)
        obj, st = graph.solve_ba(cams, pts, **dev)
        torch.cuda.synchronize()
        assert np.array_equal(cams.cpu().numpy(), ref[0]), rep
        assert np.array_equal(pts.cpu().numpy(), ref[1]), rep
        assert np.array_equal(obj.cpu().numpy(), ref[2]), rep


def test_forced_sparse_schedules_agree():
    """BLOCK (pose-block factor by elimination-tree levels, one launch),
    PERSISTENT (the whole solve in one launch with a graph queue),
    WORKGROUP (factor and solves in one workgroup per graph), HYBRID
    (per-column factor launches, workgroup solves) and SWEEPS on the same
    problem: the same tile arithmetic in different orders, so the results
    agree to rounding."""
    from paper_2207_09442_amd import Plan
    p = synth.uneven_walk_se3(batch=5, n_min=20, n_max=90, seed=22)
    poses0 = t(p["poses_init"])
    runs = [_pose_graph_run(p, Plan(p, 6, lam=0.0, solver="sparse", sparse_solve=m, device=poses0.device), poses0)
            for m in ("block", "persistent", "workgroup", "hybrid", "sweeps")]
    for r in runs[1:]:
        assert np.abs(r[0] - runs[0][0]).max() < 1e-12 * np.abs(runs[0][0]).max()
        assert r[2].tolist() == runs[0][2].tolist() == [0] * 5


def test_autotuner_picks_a_feasible_schedule_and_caches_it(tmp_path):
    from paper_2207_09442_amd import Plan
    from paper_2207_09442_amd import autotune as A
    p = synth.uneven_walk_se3(batch=4, n_min=20, n_max=60, seed=23)
    cache = str(tmp_path / "tune.json")
    best = A.autotune(p, 5, 1e-3, cache_path=cache, reps=2)
    assert best["solver"] in ("dense", "sparse") and best["ms"] > 0
    assert all(c["ms"] is not None for c in best["candidates"])     # every schedule fits this problem
    again = A.autotune(p, 5, 1e-3, cache_path=cache)
    assert again == best                                               # served from the cache
    poses0 = t(p["poses_init"])
    ref = _pose_graph_run(p, Plan(p, 5, lam=1e-3, device=poses0.device), poses0)
    got = _pose_graph_run(p, A.tuned_plan(p, 5, 1e-3, cache_path=cache), poses0)
    assert np.abs(got[0] - ref[0]).max() < 1e-10 * np.abs(ref[0]).max()


def test_ba_graph_recaptures_when_the_radii_change():
    """A captured Schur solve replays only while every argument pointer,
    the per-problem Huber radii included, is the one it was captured with:
    no radii, then radii tensor A, then tensor B (another address, other
    values) each equal the eager plan's result bit for bit."""
    from paper_2207_09442_amd import Plan
    p = synth.bundle_adjustment(batch=2, n_cams=8, n_points=50, obs_per_point=4, seed=7, pixel_sigma=2.0)
    dev = dict(obs_uv=t(p["obs_uv"]), obs_w=t(p["obs_w"]), prior_meas=t(p["prior_meas"]),
               prior_logw=t(p["prior_logw"]))
    c0, q0 = t(p["poses_init"]), t(p["points_init"])
    eager = Plan(p, 4, lam=1e-3, solver="schur", device=c0.device)
    graph = Plan(p, 4, lam=1e-3, solver="schur", device=c0.device, graph=True)
    cams_g, pts_g = c0.clone(), q0.clone()
    for radii in (None, t([1.0, 3.0]), t([2.5, 0.7])):
        cams, pts = c0.clone(), q0.clone()
        obj_e, _ = eager.solve_ba(cams, pts, huber_delta=radii, **dev)
        cams_g.copy_(c0)
        pts_g.copy_(q0)
        obj_g, _ = graph.solve_ba(cams_g, pts_g, huber_delta=radii, **dev)
        torch.cuda.synchronize()
        assert torch.equal(cams, cams_g) and torch.equal(pts, pts_g) and torch.equal(obj_e, obj_g)


def test_sparse_graph_recaptures_when_the_welsch_radii_change():
    """The same for the Welsch log-radii of the edges on the block-sparse
    solver: none, tensor A, tensor B."""
    from paper_2207_09442_amd import Plan
    p = synth.walk_se3(batch=2, n_poses=20, n_loops=10, seed=8, outliers=2)
    poses0 = t(p["poses_init"])
    dev = [t(p["edge_meas"]), t(p["edge_logw"]), t(p["prior_meas"]), t(p["prior_logw"])]
    eager = Plan(p, 5, lam=1e-3, solver="sparse", device=poses0.device)
    graph = Plan(p, 5, lam=1e-3, solver="sparse", device=poses0.device, graph=True)
    x_g = poses0.clone()
    E = len(p["edge_logw"])
    for logc in (None, t(np.full(E, 0.0)), t(np.full(E, -1.0))):
        x = poses0.clone()
        obj_e, _ = eager.solve(x, *dev, edge_logc=logc)
        x_g.copy_(poses0)
        obj_g, _ = graph.solve(x_g, *dev, edge_logc=logc)
        torch.cuda.synchronize()
        assert torch.equal(x, x_g) and torch.equal(obj_e, obj_g)
