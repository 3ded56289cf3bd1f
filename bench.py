"""Throughput of the batched DNLS inner step on one MI355X.

One step = the whole hot path over one batch: K Gauss-Newton /
Levenberg-Marquardt steps (cost evaluation, J^T J / J^T r assembly, damping,
Cholesky, triangular solves, retraction), the final undamped linearisation
that caches the factor, and the implicit backward (adjoint solve with the
cached factor and the per-cost vector-Jacobian products).

Default workload (the headline line): 128 SE(3) random-walk pose graphs of
64 poses (63 odometry edges, 64 loop closures, prior on pose 0), 10 LM steps
at lambda = 1e-3, dense 384 x 384 normal equations; float32 linearisation /
assembly with float64 factorisation and one float64 refinement sweep
(mixed), plus the same run in float64 for comparison.  --workload selects
one of the other evaluation configurations instead (SE(2) circle, 16^3
lattice on the block-sparse solver, 256 walks of 32..256 poses, bundle
adjustment on the Schur path).  Inputs are synthetic and resident in device
memory before timing starts.

Prints one JSON line.  value = graph-steps per second = B * K / (seconds per step).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DEFAULT_WORKLOAD = "se3_walk64_b128"
PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 (matrix and vector)
PEAK_HBM_GBPS = 8000.0    # MI355X HBM3E
KERNEL_SOURCES = ["paper_2207_09442_amd/csrc/dnls.hip", "paper_2207_09442_amd/csrc/dense.hpp",
                  "paper_2207_09442_amd/csrc/costs.hpp", "paper_2207_09442_amd/csrc/pose_costs.hpp",
                  "paper_2207_09442_amd/csrc/lie.hpp"]
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_dense_solve_se3_walk64_b128_traffic.txt")
MFMA_SUMMARY = os.path.join(ROOT, "profiles", "k_dense_solve_se3_walk64_b128_mfma.txt")
COST_FLOPS = 2100     # per pose-graph cost and linearisation: evaluation ~1000 + assembly ~1100
OBS_FLOPS = 340       # per reprojection cost and linearisation
BWD_COST_FLOPS = 400  # per cost in the backward (VJP)


def algorithmic_flops(problem: dict, K: int, factor_flops: float) -> tuple[float, float]:
    """(solve, backward) FLOPs the method needs (not what the kernels spend).
    Solve: K + 1 linearisations and factorisations (factor_flops each, from
    the plan's symbolic analysis) plus 2 n^2 per step for the two triangular
    solves of every dense graph; bundle adjustment adds the Schur complement
    per point (k observations: k (k + 1) / 2 camera-pair blocks at
    2 * 6 * 3 * 6 flops and k E C^-1 products at 2 * 6 * 3 * 3).  Backward:
    two triangular solves and the VJP per cost."""
    d = 6 if problem["group"] == "SE3" else 3
    B = len(problem["pose_off"]) - 1
    n_pose = np.diff(problem["pose_off"]).astype(np.float64)
    costs = np.diff(problem["edge_off"]) + np.diff(problem["prior_off"])
    n = d * n_pose
    tri = 2.0 * n ** 2
    lin = COST_FLOPS * costs.astype(np.float64)
    if "obs_off" in problem:
        obs = np.diff(problem["obs_off"]).astype(np.float64)
        k = np.bincount(problem["obs_pt"], minlength=int(problem["point_off"][-1])).astype(np.float64)
        schur = np.zeros(B)
        for b in range(B):
            kb = k[problem["point_off"][b]:problem["point_off"][b + 1]]
            schur[b] = np.sum(kb * (kb + 1) / 2 * 216 + kb * 108)
        lin = lin + OBS_FLOPS * obs + schur
        bwd_costs = costs + obs
    else:
        bwd_costs = costs
    if problem.get("_sparse"):
        tri = np.zeros(B)   # 4 nnz(L): below 0.1% of the factorisation on the lattice
    solve = (K + 1) * factor_flops + float(np.sum((K + 1) * lin + K * tri))
    backward = float(np.sum(tri + BWD_COST_FLOPS * bwd_costs))
    return solve, backward


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _summary(path: str):
    """key: value records of a committed rocprofv3 summary, or None if it is
    missing or was taken on other kernel sources."""
    try:
        with open(path) as fh:
            rec = dict(line.split(":", 1) for line in fh.read().splitlines()
                       if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    rec = {k.strip(): v.strip() for k, v in rec.items()}
    return rec if rec.get("source_hash") == kernel_hash() else None


def measured_traffic():
    """HBM bytes per launch of the mixed-precision solve kernel from the
    committed rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, scaled by
    the same counters' reading on a plain copy of known size), or None if the
    summary was taken on other kernel sources."""
    rec = _summary(TRAFFIC_SUMMARY)
    try:
        return float(rec["traffic_bytes_per_launch"]) if rec else None
    except (KeyError, ValueError):
        return None


def measured_mfma():
    """MFMA busy fraction and executed FP64 MFMA flops per launch of the
    mixed-precision solve kernel (rocprofv3 SQ counters), or None."""
    rec = _summary(MFMA_SUMMARY)
    try:
        return dict(busy_frac=float(rec["mixed_mfma_busy_frac"]),
                    executed_flops_per_launch=float(rec["mixed_mfma_flops_per_launch"])) if rec else None
    except (KeyError, ValueError):
        return None


def copy_calibration(nbytes: int, reps: int) -> None:
    """A plain device-to-device copy of nbytes, reps times: the reference
    kernel whose FETCH_SIZE / WRITE_SIZE readings calibrate the traffic
    counters (it moves exactly nbytes each way)."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}), flush=True)


def cpu_baseline(problem: dict, K: int, lam: float, n_graphs: int, passes: int):
    """The CPU oracle on the first n_graphs graphs (forward + implicit
    backward), repeated `passes` times; returns the time of all passes."""
    import torch

    from oracle import solve as S
    gs = S.graphs_of(problem)[:n_graphs]
    t0 = time.perf_counter()
    for _ in range(passes):
        res = [S.solve_graph(g, K, lam) for g in gs]
        seeds = []
        for b, r in enumerate(res):
            lo, hi = problem["pose_off"][b], problem["pose_off"][b + 1]
            _, v = S.pose_error_loss_and_seed(problem["group"], gs[0].G.to_storage(r.X).numpy(),
                                              problem["poses_gt"][lo:hi])
            seeds.append(v)
        grads = [S.implicit_grad_graph(g, r, torch.as_tensor(v),
                                       torch.zeros(g.pts.shape[0], 3, dtype=torch.float64) if g.is_ba else None)
                 for g, r, v in zip(gs, res, seeds)]
    dt = time.perf_counter() - t0
    return dt, res, seeds, grads


def progress(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD,
                    choices=["se2_circle_b1", "se3_walk64_b128", "se3_lattice16_b8", "se3_uneven_b256",
                             "ba_ring64_b4"])
    ap.add_argument("--refine", type=int, default=None,
                    help="float64 refinement sweeps of the mixed path (default: the sweeps that hold 1e-5: "
                         "2 on the 16^3 lattice, 3 on the 256-pose walks, else 1)")
    ap.add_argument("--refine-last", type=int, default=0,
                    help="mixed path: refinement sweeps in the last N steps only (N < 0: the first -N "
                         "steps; 0 = every step, the default, the one that holds 1e-5 on the gradients)")
    ap.add_argument("--sparse-solve", choices=["auto", "block", "persistent", "workgroup", "hybrid", "sweeps"],
                    default="auto", help="schedule of the block-sparse solver")
    ap.add_argument("--solver", choices=["dense", "sparse"], default=None,
                    help="override the workload's solver (bundle adjustment: sparse eliminates the points "
                         "inside the block-sparse factorisation instead of the explicit Schur complement)")
    ap.add_argument("--adaptive", action="store_true",
                    help="Levenberg-Marquardt with adaptive damping from the workload's lambda")
    ap.add_argument("--no-pair", action="store_true",
                    help="dense solver: one workgroup per graph even where a co-resident pair per graph fits")
    ap.add_argument("--dogleg", type=float, default=None, metavar="RADIUS",
                    help="Powell's dogleg with this initial trust radius")
    ap.add_argument("--backward", choices=["implicit", "dlm", "exact", "unroll"], default="implicit",
                    help="backward mode: implicit (Proposition 1), direct loss minimisation, implicit with "
                         "the exact Hessian, or unrolled through the last --unroll-steps steps (pose-graph "
                         "solvers)")
    ap.add_argument("--unroll-steps", type=int, default=None, help="truncated unrolling: steps (default all K)")
    ap.add_argument("--dlm-eps", type=float, default=1e-3)
    ap.add_argument("--sweeps", type=int, default=8, help="refinement sweeps of the exact-Hessian backward")
    ap.add_argument("--autotune", action="store_true",
                    help="pick solver, sparse solve schedule and graph capture with the autotuner "
                         "(pose graphs only; timed before the benchmark, cached)")
    ap.add_argument("--cpu-graphs", type=int, default=None,
                    help="graphs in the CPU oracle sample (default: the whole batch of the headline "
                         "workload, a few graphs otherwise)")
    ap.add_argument("--cpu-passes", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (traffic-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(graphs are independent, so a multi-GPU run would shard the batch with no "
              "communication; the library runs on one device).", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration(args.copy_calibration, max(1, args.steps))
        return

    import torch

    import synth
    from paper_2207_09442_amd import Plan, project_grad

    dev = torch.device("cuda:0")
    W = synth.WORKLOADS[args.workload]
    K, lam, solver = W["iterations"], W["lam"], W["solver"]
    if args.refine is None:
        # the sweeps that hold every result within 1e-5: more on the worse
        # conditioned workloads (cond(H) ~4e8 walks, ~7e8 lattice, ~1e11
        # for the 256-pose walks)
        args.refine = {"se3_lattice16_b8": 2, "se3_uneven_b256": 3}.get(args.workload, 1)
    ba = solver == "schur"
    if args.solver and not ba:
        solver = args.solver
    elif args.solver == "sparse" and ba:
        solver = "sparse"      # bundle adjustment with the points eliminated inside the sparse factorisation
    p = W["fn"](**W["kwargs"])
    if ba and args.backward not in ("implicit", "dlm"):
        raise SystemExit(f"--backward {args.backward}: the Schur solver has the implicit and DLM backward modes")
    B = len(p["pose_off"]) - 1
    t = lambda x: torch.as_tensor(np.asarray(x), dtype=torch.float64, device=dev).contiguous()
    init, gt = t(p["poses_init"]), t(p["poses_gt"])
    if ba:
        aux = dict(obs_uv=t(p["obs_uv"]), obs_w=t(p["obs_w"]), prior_meas=t(p["prior_meas"]),
                   prior_logw=t(p["prior_logw"]))
        pts_init = t(p["points_init"])
    else:
        aux = (t(p["edge_meas"]), t(p["edge_logw"]), t(p["prior_meas"]), t(p["prior_logw"]))

    schedule = dict(sparse_solve=args.sparse_solve, graph=False, adaptive=bool(args.adaptive), dogleg=args.dogleg,
                    keep_iterates=args.backward == "unroll", pair=not args.no_pair)
    if args.autotune and not ba:
        from paper_2207_09442_amd.autotune import autotune
        best = autotune(p, K, lam, precision=W["precision"], refine=args.refine if W["precision"] == "mixed" else 0,
                        device=dev)
        solver = best["solver"]
        schedule = dict(sparse_solve=best["sparse_solve"], graph=best["graph"], adaptive=bool(args.adaptive),
                        dogleg=args.dogleg, keep_iterates=args.backward == "unroll", pair=best.get("pair", False))
        progress(f"autotuned schedule: {solver} {schedule} ({best['ms']:.3f} ms)")

    def run(precision: str, refine: int):
        plan = Plan(p, K, lam=lam, solver=solver, precision=precision, refine=refine, device=dev,
                    refine_last=args.refine_last if precision == "mixed" else 0, **schedule)
        poses = init.clone()
        pts = pts_init.clone() if ba else None

        def solve():
            return plan.solve_ba(poses, pts, **aux) if ba else plan.solve(poses, *aux)

        # seed: tangent gradient of L = sum ||X - X_gt||^2 on the storage at the
        # warm-up solution (an input of the backward, fixed during timing)
        solve()
        seed = project_grad(p["group"], poses.reshape(plan.V, -1), (2 * (poses - gt)).reshape(plan.V, -1))

        def backward(st):
            if ba:
                return plan.backward_ba(poses, pts, status=st, seed_cam=seed, mode=args.backward, eps=args.dlm_eps,
                                        **aux)
            return plan.backward(poses, *aux, st, seed, mode=args.backward, eps=args.dlm_eps, sweeps=args.sweeps,
                                 steps=args.unroll_steps)

        stream = torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        fwd_ms, bwd_ms = [], []

        def one_step(record: bool):
            poses.copy_(init)
            if ba:
                pts.copy_(pts_init)
            if record:
                ev[0].record(stream)
            obj, st = solve()
            if record:
                ev[1].record(stream)
            out = backward(st)
            if record:
                ev[2].record(stream)
            return obj, st, out

        for _ in range(args.warmup):
            one_step(False)
        torch.cuda.synchronize()
        progress(f"{precision}: warm-up done")
        # per-step events (solve and backward separately; one host sync per step)
        for _ in range(args.steps):
            one_step(True)
            torch.cuda.synchronize()
            fwd_ms.append(ev[0].elapsed_time(ev[1]))
            bwd_ms.append(ev[1].elapsed_time(ev[2]))
        progress(f"{precision}: per-step events done, solve {np.mean(fwd_ms):.3f} ms")
        # the timed loop: K steps back to back, synchronised on both sides
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            obj, st, out = one_step(False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        progress(f"{precision}: timed loop done, {1e3 * wall / args.steps:.3f} ms/step")
        return dict(plan=plan, poses=poses.cpu().numpy(), points=pts.cpu().numpy() if ba else None,
                    status=st.cpu().numpy(),
                    grads={k: v.cpu().numpy() for k, v in out.items()}, ms_step=1e3 * wall / args.steps,
                    fwd_ms=float(np.mean(fwd_ms)), bwd_ms=float(np.mean(bwd_ms)))

    main_prec = W["precision"]
    runs = {}
    if main_prec == "mixed":
        runs["mixed"] = run("mixed", args.refine)
    runs["fp64"] = run("fp64", 0)
    head = runs[main_prec]
    graph_steps = B * K
    value = graph_steps / (head["ms_step"] * 1e-3)
    f_alg, f_exec = head["plan"].flops()
    if solver == "sparse":
        p["_sparse"] = True
    solve_flops, bwd_flops = algorithmic_flops(p, K, f_alg)
    p.pop("_sparse", None)
    achieved = solve_flops / (head["fwd_ms"] * 1e-3) / 1e12
    single_kernel = solver == "dense"
    head_default = args.workload == DEFAULT_WORKLOAD and solver == "dense" and main_prec == "mixed"
    pair_used = single_kernel and head["plan"].pair_active()
    kernel = ("k_dense_solve<%d, %s, false, %s>" % (3 if p["group"] == "SE3" else 2,
                                                     "true" if main_prec == "mixed" else "false",
                                                     "true" if pair_used else "false")
              if single_kernel else "solve (all kernels of dnls_solve)")
    cfg = {"workload": args.workload, "batch": B, "iterations": K,
           "optimizer": W["optimizer"], "lambda": lam, "precision": main_prec,
           "refine": args.refine if main_prec == "mixed" else 0,
           "refine_last": args.refine_last if main_prec == "mixed" else 0, "solver": solver,
           "schedule": dict(schedule, autotuned=bool(args.autotune and not ba)),
           "backward": {"implicit": "implicit", "dlm": f"dlm (eps={args.dlm_eps:g})",
                        "exact": f"exact Hessian ({args.sweeps} sweeps)",
                        "unroll": f"unrolled ({args.unroll_steps or K} of {K} steps)"}[args.backward]}
    if args.workload == "se3_walk64_b128":
        cfg.update(poses=64, loop_closures=64)
    line = {
        "metric": "GN/LM steps/sec incl. implicit-diff backward, mixed vs FP64 at 1e-5 rel err",
        "value": value,
        "unit": "graph-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if main_prec == "mixed" else "f64",
        "data": "synthetic",
        "config": cfg,
        "breakdown": {"solve_ms": head["fwd_ms"], "backward_ms": head["bwd_ms"]},
        "roofline": {"bound": "mfma", "kernel": kernel, "achieved": achieved,
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": measured_traffic() if head_default else None,
                     "mfma_counters": measured_mfma() if head_default else None,
                     "algorithmic_flops_per_launch": solve_flops,
                     "factor_flops_algorithmic": f_alg, "factor_flops_executed": f_exec},
    }
    traffic = line["roofline"]["traffic"]
    if traffic:
        # measured HBM bytes of the launch over its live duration, against the 8 TB/s peak
        hbm = traffic / (head["fwd_ms"] * 1e-3) / 1e9
        line["roofline"]["hbm_GBps"] = hbm
        line["roofline"]["hbm_frac"] = hbm / PEAK_HBM_GBPS
    if main_prec == "mixed":
        f = runs["fp64"]
        line["fp64"] = {"value": graph_steps / (f["ms_step"] * 1e-3), "ms_per_step": f["ms_step"],
                        "solve_ms": f["fwd_ms"], "backward_ms": f["bwd_ms"]}
    if args.workload == "se2_circle_b1":
        line["us_per_graph_step"] = 1e3 * head["ms_step"] / K
        # latency floor: one replay of a captured graph with one trivial kernel
        line["empty_graph_replay_us"] = empty_graph_replay_us()
    # the oracle's sparse path on a 4096-pose lattice takes minutes per graph: no CPU sample there
    default_cpu = {"se3_walk64_b128": 128, "se2_circle_b1": 1, "se3_uneven_b256": 32,
                   "ba_ring64_b4": 4, "se3_lattice16_b8": 0}[args.workload]
    ng = min(B, default_cpu if args.cpu_graphs is None else args.cpu_graphs)
    # the CPU sample and the error check are of the implicit backward
    if not args.no_cpu and ng > 0 and args.backward == "implicit":
        progress(f"CPU oracle on {ng} graph(s)")
        import torch as _t
        npass = max(1, args.cpu_passes)
        dt, res, seeds, grads = cpu_baseline(p, K, lam, ng, npass)
        line["cpu_baseline"] = {"value": npass * ng * K / dt, "unit": "graph-steps/s",
                                "cores": _t.get_num_threads(), "kind": "oracle",
                                "sample": f"{npass} pass(es) over the first {ng} of the {B} graphs, forward "
                                          f"(K={K}) + implicit backward, {dt:.1f} s"}
        # the same sample on one thread (a bounded part of it: a quarter of the graphs, one pass)
        ng1 = max(1, ng // 4)
        nthreads = _t.get_num_threads()
        _t.set_num_threads(1)
        dt1, _, _, _ = cpu_baseline(p, K, lam, ng1, 1)
        _t.set_num_threads(nthreads)
        line["cpu_baseline_1thread"] = {"value": ng1 * K / dt1, "unit": "graph-steps/s", "cores": 1,
                                        "kind": "oracle",
                                        "sample": f"1 pass over the first {ng1} graph(s), {dt1:.1f} s"}
        if ba:
            line["error_vs_oracle"] = errors_vs_oracle_ba(p, runs, res, seeds, grads, aux, ng, t, dev)
        else:
            line["error_vs_oracle"] = errors_vs_oracle(p, runs, res, seeds, grads, aux, ng, t, dev)
    elif not args.no_cpu and args.workload == "se3_lattice16_b8" and args.backward == "implicit":
        import torch as _t
        progress("CPU oracle (sparse) on one Gauss-Newton step of graph 0")
        dt = cpu_baseline_sparse(p)
        line["cpu_baseline"] = {"value": 1.0 / dt, "unit": "graph-steps/s", "cores": _t.get_num_threads(),
                                "kind": "oracle",
                                "sample": f"one Gauss-Newton step of graph 0 (linearisation, SuperLU "
                                          f"factorisation, solve, retraction), {dt:.1f} s; the final "
                                          f"linearisation and backward not included"}
    print(json.dumps(line), flush=True)


def _ew(a, b, floor, scale=None):
    """max_i |a_i - b_i| / max(|b_i|, floor * scale), scale = max |b| by default."""
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    sc = float(np.abs(b).max()) if scale is None else float(scale)
    den = np.maximum(np.abs(b), floor * sc)
    return float(np.max(np.abs(a - b) / np.where(den > 0, den, 1.0))) if b.size else 0.0


def _spread(g, r, v, pose_rel):
    """The oracle's own gradient spread on one graph under rounding-level
    changes (permuted summation of the final linearisation; theta_K moved by
    pose_rel): max-norm change over the gradient's max norm."""
    import dataclasses

    import torch

    from oracle import solve as S
    rng = np.random.default_rng(0)
    vt = torch.as_tensor(v, dtype=torch.float64)
    flat = lambda o, inv=slice(None): np.concatenate([o["edge_logw"].detach().numpy()[inv],
                                                      o["tau"].detach().numpy()[inv].ravel(),
                                                      o["prior_logw"].detach().numpy()])
    ref = flat(S.implicit_grad_graph(g, r, vt))
    perm = rng.permutation(len(g.ei))
    pt = torch.as_tensor(perm)
    gp = dataclasses.replace(g, ei=g.ei[pt], ej=g.ej[pt], Z=g.Z[pt], logw_e=g.logw_e[pt])
    lin = S.linearize_pose_graph(gp, r.X)
    a = flat(S.implicit_grad_graph(gp, dataclasses.replace(r, lin=lin, factor=(torch.linalg.cholesky(lin.H),)), vt),
             np.argsort(perm))
    st = g.G.to_storage(r.X)
    xi = torch.as_tensor(rng.normal(size=(r.X.shape[0], g.G.dof)), dtype=torch.float64)
    X2 = g.G.retract(r.X, xi / xi.norm() * max(pose_rel, 1e-14) * float(st.norm()))
    lin2 = S.linearize_pose_graph(g, X2)
    b = flat(S.implicit_grad_graph(g, dataclasses.replace(r, X=X2, lin=lin2,
                                                          factor=(torch.linalg.cholesky(lin2.H),)), vt))
    return max(np.abs(a - ref).max(), np.abs(b - ref).max()) / max(float(np.abs(ref).max()), 1e-300)


def errors_vs_oracle(p, runs, res, seeds, grads, aux, ng, t, dev):
    """Errors of the GPU runs against the oracle on the sampled graphs (the
    backward rerun with the oracle's seeds): per graph, relative norms of the
    poses and of the gradient (log-weights, tangents, prior log-weights),
    element-wise ratios (poses: floor 1e-3 of the graph's largest entry;
    gradients: against the graph's largest gradient element in float64,
    floor 1e-3 of it in mixed), and for float64 the largest ratio of the
    gradient error to its tolerance max(1e-10, 3 s), s the oracle's own
    spread on that graph."""
    import torch

    from oracle import lie
    from oracle import solve as S
    grp = lie.SE3 if p["group"] == "SE3" else lie.SE2
    d = 6 if p["group"] == "SE3" else 3
    gs = S.graphs_of(p)
    errs = {}
    for name, r in runs.items():
        e = dict(pose_rel_err_max=0.0, pose_ew_max=0.0, grad_rel_err_max=0.0, grad_ew_max=0.0)
        if name == "fp64":
            e["grad_err_over_tolerance_max"] = 0.0
        full = np.zeros((p["pose_off"][-1], d))
        for b in range(ng):
            full[p["pose_off"][b]:p["pose_off"][b + 1]] = seeds[b]
        st_dev = torch.as_tensor(r["status"], device=dev)
        gr = r["plan"].backward(t(r["poses"]), *aux, st_dev, t(full))
        gr = {k: v.cpu().numpy() for k, v in gr.items()}
        for b in range(ng):
            lo, hi = p["pose_off"][b], p["pose_off"][b + 1]
            e0, e1 = p["edge_off"][b], p["edge_off"][b + 1]
            q0, q1 = p["prior_off"][b], p["prior_off"][b + 1]
            ref = grp.to_storage(res[b].X).numpy()
            prel = np.linalg.norm(r["poses"][lo:hi] - ref) / np.linalg.norm(ref)
            e["pose_rel_err_max"] = max(e["pose_rel_err_max"], prel)
            e["pose_ew_max"] = max(e["pose_ew_max"], _ew(r["poses"][lo:hi], ref, 1e-3))
            mine = [gr["edge_logw"][e0:e1], gr["edge_tau"][e0:e1].ravel(), gr["prior_logw"][q0:q1]]
            theirs = [grads[b]["edge_logw"].detach().numpy(), grads[b]["tau"].detach().numpy().ravel(),
                      grads[b]["prior_logw"].detach().numpy()]
            a, c = np.concatenate(mine), np.concatenate(theirs)
            e["grad_rel_err_max"] = max(e["grad_rel_err_max"], np.linalg.norm(a - c) / np.linalg.norm(c))
            scale = float(np.abs(c).max())
            ew = max(_ew(m, x, 1e-3 if name == "mixed" else 1.0, scale) for m, x in zip(mine, theirs))
            e["grad_ew_max"] = max(e["grad_ew_max"], ew)
            if name == "fp64":
                tol = 1e-10 if ew < 1e-10 else max(1e-10, 3.0 * _spread(gs[b], res[b], seeds[b], prel))
                e["grad_err_over_tolerance_max"] = max(e["grad_err_over_tolerance_max"], ew / tol)
        errs[name] = e
    return errs


def errors_vs_oracle_ba(p, runs, res, seeds, grads, aux, ng, t, dev):
    """Bundle adjustment: errors of the GPU runs against the oracle on the
    sampled problems (cameras, points, and the gradients of the observation
    weights, prior log-weights and per-observation radii, the backward rerun
    with the oracle's camera seeds and zero point seeds): relative norms per
    problem and element-wise ratios as for pose graphs."""
    import torch

    from oracle import lie
    errs = {}
    for name, r in runs.items():
        e = dict(cam_rel_err_max=0.0, cam_ew_max=0.0, point_rel_err_max=0.0, point_ew_max=0.0,
                 grad_rel_err_max=0.0, grad_ew_max=0.0)
        sc = np.zeros((p["pose_off"][-1], 6))
        for b in range(ng):
            sc[p["pose_off"][b]:p["pose_off"][b + 1]] = seeds[b]
        st_dev = torch.as_tensor(r["status"], device=dev)
        gr = r["plan"].backward_ba(t(r["poses"]), t(r["points"]), status=st_dev, seed_cam=t(sc), **aux)
        gr = {k: v.cpu().numpy() for k, v in gr.items()}
        for b in range(ng):
            c0, c1 = p["pose_off"][b], p["pose_off"][b + 1]
            q0, q1 = p["point_off"][b], p["point_off"][b + 1]
            o0, o1 = p["obs_off"][b], p["obs_off"][b + 1]
            r0, r1 = p["prior_off"][b], p["prior_off"][b + 1]
            cref = lie.SE3.to_storage(res[b].X).numpy()
            pref = res[b].pts.numpy()
            e["cam_rel_err_max"] = max(e["cam_rel_err_max"],
                                       np.linalg.norm(r["poses"][c0:c1] - cref) / np.linalg.norm(cref))
            e["cam_ew_max"] = max(e["cam_ew_max"], _ew(r["poses"][c0:c1], cref, 1e-3))
            e["point_rel_err_max"] = max(e["point_rel_err_max"],
                                         np.linalg.norm(r["points"][q0:q1] - pref) / np.linalg.norm(pref))
            e["point_ew_max"] = max(e["point_ew_max"], _ew(r["points"][q0:q1], pref, 1e-3))
            mine = [gr["obs_w"][o0:o1], gr["prior_logw"][r0:r1], gr["obs_delta"][o0:o1]]
            theirs = [grads[b][k].detach().numpy() for k in ("obs_w", "prior_logw", "obs_delta")]
            a, c = np.concatenate(mine), np.concatenate(theirs)
            e["grad_rel_err_max"] = max(e["grad_rel_err_max"], np.linalg.norm(a - c) / np.linalg.norm(c))
            scale = float(np.abs(c).max())
            e["grad_ew_max"] = max(e["grad_ew_max"], max(_ew(m, x, 1e-3 if name == "mixed" else 1.0, scale)
                                                         for m, x in zip(mine, theirs)))
        errs[name] = e
    return errs


def cpu_baseline_sparse(p):
    """The oracle's sparse path on graph 0 of the lattice, one Gauss-Newton
    step (linearisation, sparse factorisation, solve, retraction): the
    bounded sample of the block-sparse workload, whose full K + 1
    factorisations per graph take minutes on the CPU."""
    import torch

    from oracle import solve as S
    g = S.graphs_of(p)[0]
    t0 = time.perf_counter()
    s, H, gv = S.linearize_pose_graph_sparse(g, g.X)
    lu = S._sparse_factor(H)
    delta = torch.as_tensor(lu.solve(gv), dtype=torch.float64)
    g.G.retract(g.X, -delta.reshape(-1, g.G.dof))
    return time.perf_counter() - t0


def empty_graph_replay_us(reps: int = 200) -> float:
    """Time of one replay of a captured HIP graph holding a single trivial
    kernel (one float64 element incremented): the launch floor against which
    the latency-bound one-graph workload is read."""
    import torch
    x = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        x.add_(1.0)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        x.add_(1.0)
    for _ in range(10):
        g.replay()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        g.replay()
    b.record()
    torch.cuda.synchronize()
    return 1e3 * a.elapsed_time(b) / reps


if __name__ == "__main__":
    main()
