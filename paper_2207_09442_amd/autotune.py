"""Schedule autotuner: picks the solver (dense per-graph kernel, on one
workgroup or a co-resident pair per graph, or block-sparse tiles), the sparse schedule (factorisation and triangular
solves in one workgroup per graph, per-column launches, or per-column
factorisation with workgroup solves) and HIP-graph capture for a problem
structure by
timing every feasible candidate on the device, forward and implicit backward
together.  Results are cached in a JSON file keyed by a hash of the
structure and the optimizer settings, so a structure is tuned once.

The candidates run the real kernels through the C ABI on the caller's data;
nothing here changes what is computed, only how it is scheduled (every
candidate matches the oracle to the tolerances of the parity tests).
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

CACHE_ENV = "DNLS_AUTOTUNE_CACHE"
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "dnls_autotune.json")

CANDIDATES = [
    dict(solver="dense", sparse_solve="auto", graph=False),
    dict(solver="dense", sparse_solve="auto", graph=False, pair=True),
    dict(solver="sparse", sparse_solve="block", graph=False),
    dict(solver="sparse", sparse_solve="persistent", graph=False),
    dict(solver="sparse", sparse_solve="workgroup", graph=False),
    dict(solver="sparse", sparse_solve="workgroup", graph=True),
    dict(solver="sparse", sparse_solve="hybrid", graph=False),
    dict(solver="sparse", sparse_solve="hybrid", graph=True),
    dict(solver="sparse", sparse_solve="sweeps", graph=False),
    dict(solver="sparse", sparse_solve="sweeps", graph=True),
]


def structure_key(problem: dict, iterations: int, lam: float, precision: str, refine: int) -> str:
    """Hash of everything that determines the schedule's cost: the graph
    structure (offsets, edge and prior incidence), the group and the
    optimizer settings, plus the device name."""
    import torch
    h = hashlib.sha256()
    for k in ("pose_off", "edge_off", "prior_off", "edge_ij", "prior_var"):
        h.update(np.ascontiguousarray(np.asarray(problem[k], dtype=np.int32)).tobytes())
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
    h.update(json.dumps([problem["group"], int(iterations), float(lam), precision, int(refine), dev]).encode())
    return h.hexdigest()[:24]


def _load(path: str) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(path: str, cache: dict) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_candidate(problem, iterations, lam, precision, refine, cand, reps, device):
    """Median milliseconds of solve + backward for one candidate, or None if
    the plan rejects it (e.g. a graph too large for the workgroup solve)."""
    import torch

    from . import DnlsError, Plan, project_grad
    try:
        plan = Plan(problem, iterations, lam=lam, precision=precision, refine=refine, device=device, **cand)
    except DnlsError:
        return None
    t = lambda x: torch.as_tensor(np.asarray(x), dtype=torch.float64, device=device).contiguous()
    init = t(problem["poses_init"])
    aux = (t(problem["edge_meas"]), t(problem["edge_logw"]), t(problem["prior_meas"]), t(problem["prior_logw"]))
    poses = init.clone()
    _, st = plan.solve(poses, *aux)
    seed = project_grad(problem["group"], poses.reshape(plan.V, -1), poses.reshape(plan.V, -1))
    times = []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for r in range(reps + 1):
        poses.copy_(init)
        ev0.record()
        _, st = plan.solve(poses, *aux)
        plan.backward(poses, *aux, st, seed)
        ev1.record()
        torch.cuda.synchronize()
        if r > 0:
            times.append(ev0.elapsed_time(ev1))
    return float(np.median(times))


def autotune(problem: dict, iterations: int, lam: float = 0.0, precision: str = "fp64", refine: int = 0,
             device: str = "cuda", reps: int = 3, cache_path: str | None = None, force: bool = False) -> dict:
    """Best schedule for a pose-graph problem: a dict of Plan keyword
    arguments (solver, sparse_solve, graph) plus the measured times of all
    candidates.  Bundle adjustment has a single (Schur) schedule and is not
    tuned."""
    if "point_off" in problem:
        raise ValueError("bundle adjustment has a single schedule (solver='schur')")
    path = cache_path or os.environ.get(CACHE_ENV, DEFAULT_CACHE)
    key = structure_key(problem, iterations, lam, precision, refine)
    cache = _load(path)
    if not force and key in cache:
        return cache[key]
    t0 = time.perf_counter()
    timings = []
    for cand in CANDIDATES:
        ms = _time_candidate(problem, iterations, lam, precision, refine, cand, reps, device)
        timings.append(dict(cand, ms=ms))
    feasible = [c for c in timings if c["ms"] is not None]
    best = min(feasible, key=lambda c: c["ms"])
    result = dict(solver=best["solver"], sparse_solve=best["sparse_solve"], graph=best["graph"],
                  pair=bool(best.get("pair", False)), ms=best["ms"], candidates=timings,
                  tuning_seconds=time.perf_counter() - t0)
    cache[key] = result
    _store(path, cache)
    return result


def tuned_plan(problem: dict, iterations: int, lam: float = 0.0, precision: str = "fp64", refine: int = 0,
               device: str = "cuda", **kw):
    """Plan with the autotuned schedule."""
    from . import Plan
    best = autotune(problem, iterations, lam, precision, refine, device, **kw)
    return Plan(problem, iterations, lam=lam, precision=precision, refine=refine, device=device,
                solver=best["solver"], sparse_solve=best["sparse_solve"], graph=best["graph"],
                pair=best.get("pair", False))
