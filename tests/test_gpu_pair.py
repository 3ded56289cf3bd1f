"""GPU parity of the two-workgroups-per-graph dense schedule
(DNLS_FLAG_PAIR: a co-resident pair of workgroups shares every
factorisation, synchronised through device-memory event counters) against
the oracle and against the one-workgroup kernel, through the C ABI: the
full 128-graph workload (where the pair fits), ragged batches with weights
and tangents, mixed precision, adaptive damping, failed graphs, and the
implicit backward on the factor the pair wrote."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import synth
from oracle import solve as S

from gpu_util import oracle_grad_at, oracle_grads, oracle_solve, rel, stationary_equivalent, t

pytestmark = pytest.mark.gpu
rng = np.random.default_rng(7070)


def _solve(p, K, lam, pair, precision="fp64", refine=0, tau=None, adaptive=False):
    from paper_2207_09442_amd import Plan
    plan = Plan(p, K, lam=lam, precision=precision, refine=refine, device="cuda", adaptive=adaptive, pair=pair)
    poses = t(p["poses_init"])
    aux = (t(p["edge_meas"]), t(p["edge_logw"]), t(p["prior_meas"]), t(p["prior_logw"]))
    tau_d = None if tau is None else t(tau)
    obj, st = plan.solve(poses, *aux, edge_tau=tau_d)
    torch.cuda.synchronize()
    return plan, poses, obj, st, aux, tau_d


def _check(p, K, lam, graphs=None, tol=1e-10, precision="fp64", refine=0, tau=None, adaptive=False):
    plan, poses, obj, st, aux, tau_d = _solve(p, K, lam, True, precision, refine, tau, adaptive)
    assert plan.schedule()["pair"]          # every batch here leaves room for two workgroups per graph
    _, poses1, obj1, st1, _, _ = _solve(p, K, lam, False, precision, refine, tau, adaptive)
    got = poses.cpu().numpy()
    # same algorithm on two schedules: equal up to the rounding of the split factorisation
    assert np.array_equal(st.cpu().numpy(), st1.cpu().numpy())
    assert rel(got, poses1.cpu().numpy()) < 1e-12
    B = len(p["pose_off"]) - 1
    graphs = list(range(B)) if graphs is None else graphs
    gs, res = oracle_solve(p, K, lam, tau=tau, graphs=graphs, adaptive=adaptive)
    seeds = [rng.normal(size=(int(p["pose_off"][b + 1] - p["pose_off"][b]), 6)) for b in graphs]
    full = np.zeros((int(p["pose_off"][-1]), 6))
    for gi, b in enumerate(graphs):
        full[p["pose_off"][b]:p["pose_off"][b + 1]] = seeds[gi]
    gr = plan.backward(poses, *aux, st, t(full), edge_tau=tau_d)
    gr = {k: v.cpu().numpy() for k, v in gr.items()}
    ref = oracle_grads(gs, res, seeds)
    ob = obj.cpu().numpy()
    for gi, b in enumerate(graphs):
        lo, hi = int(p["pose_off"][b]), int(p["pose_off"][b + 1])
        e0, e1 = int(p["edge_off"][b]), int(p["edge_off"][b + 1])
        assert st[b] == res[gi].status == S.OK
        ep = rel(got[lo:hi], gs[gi].G.to_storage(res[gi].X).numpy())
        if ep >= tol and precision == "fp64" and adaptive:
            # adaptive damping at the rounding floor: a trial step whose
            # objective change is within the rounding of S is accepted or
            # rejected by rounding alone, on either side; the GPU's theta_K
            # must then be the oracle's iterate after some j < K steps, with
            # the oracle's later steps all at that floor
            S_K = float(res[gi].lin.S)
            match = []
            for j in range(K - 1, 0, -1):
                rj = S.solve_graph(gs[gi], j, lam, tau=gs[gi].tau, adaptive=True)
                Sj = float(S.linearize_pose_graph(gs[gi], rj.X, tau=gs[gi].tau).S)
                if abs(Sj - S_K) > 1e-13 * S_K:
                    break
                if rel(got[lo:hi], gs[gi].G.to_storage(rj.X).numpy()) < tol:
                    match.append(j)
            print(f"\n  graph {b}: poses {ep:.2e} from the oracle's theta_K; equal to its iterate after "
                  f"{match} steps, whose later steps change S by less than 1e-13")
            assert match, (b, ep)
        elif ep >= tol and precision == "fp64":
            # a float64 iteration converged to the rounding floor of its
            # gradient fixes theta_K only up to that floor: the GPU's iterate
            # must be as stationary as the oracle's
            ok, n_gpu, n_ref, ds = stationary_equivalent(gs[gi], res[gi], got[lo:hi])
            print(f"\n  graph {b}: poses {ep:.2e} apart; oracle gradient norm {n_gpu:.2e} at the GPU's "
                  f"theta_K, {n_ref:.2e} at its own; objectives {ds:.1e} apart")
            assert ok, (b, ep, n_gpu, n_ref, ds)
        else:
            assert ep < tol, (b, ep)
        assert rel(ob[b], np.asarray(res[gi].objective)) < max(tol, 1e-12) * (1e3 if precision == "mixed" else 1)
        mine = np.concatenate([gr["edge_logw"][e0:e1], gr["edge_tau"][e0:e1].ravel()])
        theirs = np.concatenate([ref[gi]["edge_logw"], ref[gi]["tau"].ravel()])
        if ep >= tol and precision == "fp64":
            # theta_K taken by the reading above: the backward is compared at
            # the GPU's theta_K (the oracle's gradient there, same seed)
            sh = oracle_grad_at(gs[gi], res[gi], got[lo:hi], seeds[gi])
            theirs = np.concatenate([sh["edge_logw"], sh["tau"].ravel()])
        ev = np.linalg.eigvalsh(res[gi].lin.H.numpy())
        assert rel(mine, theirs) < max(tol, 0.5 * (ev[-1] / ev[0]) * np.finfo(np.float64).eps)


def test_pair_walk64_b128_fp64_and_mixed():
    p = synth.walk_se3(batch=128)
    _check(p, 10, 1e-3, graphs=[0, 37, 81, 127])
    _check(p, 10, 1e-3, graphs=[0, 127], precision="mixed", refine=1, tol=1e-5)


def test_pair_ragged_with_weights_and_tau():
    p = synth.uneven_walk_se3(batch=6, n_min=3, n_max=60, seed=71)
    p["edge_logw"] = rng.normal(scale=0.3, size=len(p["edge_logw"]))
    tau = 0.01 * rng.normal(size=(len(p["edge_logw"]), 6))
    _check(p, 6, 1e-3, tau=tau)


def test_pair_adaptive():
    p = synth.walk_se3(batch=4, n_poses=20, n_loops=12, seed=72)
    _check(p, 8, 1e-2, adaptive=True)


def test_pair_failed_graphs_are_frozen():
    p = synth.walk_se3(batch=3, n_poses=24, n_loops=8, seed=17)
    last = int(p["pose_off"][1]) + 23
    keep = ~((p["edge_ij"][:, 0] == last) | (p["edge_ij"][:, 1] == last))
    counts = [int(keep[p["edge_off"][b]:p["edge_off"][b + 1]].sum()) for b in range(3)]
    p["edge_ij"], p["edge_meas"], p["edge_logw"] = p["edge_ij"][keep], p["edge_meas"][keep], p["edge_logw"][keep]
    p["edge_off"] = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    p["edge_meas"] = p["edge_meas"].copy()
    p["edge_meas"][p["edge_off"][2] + 1, 0, 3] = np.nan
    plan, poses, obj, st, _, _ = _solve(p, 5, 0.0, True)
    assert plan.schedule()["pair"]
    assert st.cpu().tolist() == [0, 1, 2]
    got = poses.cpu().numpy()
    for b in (1, 2):
        lo, hi = p["pose_off"][b], p["pose_off"][b + 1]
        assert np.array_equal(got[lo:hi], p["poses_init"][lo:hi])


def test_pair_gives_up_without_hanging(monkeypatch):
    """Failure handling forced from the host: with a poll limit of one
    (DNLS_PAIR_SPIN=1) the workgroups of a graph stop waiting for each other
    almost at once; every kernel still exits, and a graph that gave up
    reports DNLS_GRAPH_TIMEOUT (3) on both schedules that share a
    factorisation."""
    monkeypatch.setenv("DNLS_PAIR_SPIN", "1")
    p = synth.walk_se3(batch=16)
    _, poses, obj, st, _, _ = _solve(p, 3, 1e-3, True)
    codes = set(st.cpu().tolist())
    assert codes <= {S.OK, 3} and 3 in codes
    from paper_2207_09442_amd import Plan
    q = synth.bundle_adjustment(batch=2, n_cams=16, n_points=80, obs_per_point=4, seed=4)
    plan = Plan(q, 3, lam=1e-3, solver="schur", device="cuda", pair=True)
    assert plan.schedule()["pair"]
    _, stb = plan.solve_ba(t(q["poses_init"]), t(q["points_init"]), obs_uv=t(q["obs_uv"]), obs_w=t(q["obs_w"]),
                           prior_meas=t(q["prior_meas"]), prior_logw=t(q["prior_logw"]))
    torch.cuda.synchronize()
    codes = set(stb.cpu().tolist())
    assert codes <= {S.OK, 3} and 3 in codes


def test_pair_deep_panel_chains():
    """Graphs of 178 and 108 poses in one launch (npad 1088 and 704: 17 and
    11 panels, so the look-ahead chain, the tiles of the panel before the
    diagonal one and the inverse reloads run many times on both roles, with
    two panel counts): the pair matches one workgroup per graph to the
    rounding of the split factorisation, and the oracle on the smaller
    graph."""
    p = synth.uneven_walk_se3(batch=2, n_min=100, n_max=180, seed=93)
    assert list(np.diff(p["pose_off"])) == [178, 108]
    _check(p, 4, 1e-3, graphs=[1])


def test_pair_not_used_for_one_panel():
    """With every graph within one 64-wide panel the follower would have no
    row group: the plan keeps one workgroup per graph (the schedule query
    says so) and the solve is the one-workgroup kernel's."""
    p = synth.circle_se2(batch=2, n_poses=16, n_loops=8, seed=3)
    plan, poses, obj, st, _, _ = _solve(p, 4, 0.0, True)
    assert not plan.schedule()["pair"]
    _, poses1, _, st1, _, _ = _solve(p, 4, 0.0, False)
    assert np.array_equal(poses.cpu().numpy(), poses1.cpu().numpy())
