"""Python binding of the MI355X DNLS library (ctypes over include/dnls.h).

Argument marshalling only: every step of the inner loop and of the implicit
backward runs in the HIP kernels of libdnls.so; PyTorch provides device
memory and the stream.  The library must have been built (see build.py);
importing works without it, but any call raises if it is missing.

Objects follow the paper's problem statement (Section 3): a batch of
objectives given by variables (poses), cost functions (relative-pose and
prior costs with their measurements) and scalar cost weights (log-weights),
an optimizer (Gauss-Newton, or Levenberg-Marquardt with a fixed damping)
and the implicit backward mode (Section 4.3).
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref

import numpy as np

__all__ = ["lib", "Plan", "DNLSFunction", "Layer", "project_grad", "DnlsError", "LIB_PATH"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdnls.so")

SOLVERS = {"dense": 0, "schur": 1, "sparse": 2}
PRECISIONS = {"fp64": 0, "mixed": 1}
SPARSE_SOLVES = {"auto": 0, "workgroup": 1, "sweeps": 2, "hybrid": 3, "persistent": 4, "block": 5}
BACKWARD_MODES = {"implicit": 0, "dlm": 1, "exact": 2, "unroll": 3}
FLAG_GRAPH = 1
FLAG_ADAPTIVE_LM = 2
FLAG_DOGLEG = 4
FLAG_KEEP_ITERATES = 8
FLAG_PAIR = 16
GROUPS = {"SE2": 2, "SE3": 3}
STATUS = {0: "ok", 1: "not_pd", 2: "nonfinite"}

_i32p = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p


class DnlsError(RuntimeError):
    pass


class _Problem(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("group", ctypes.c_int32),
                ("pose_off", _i32p), ("edge_off", _i32p), ("edge_ij", _i32p),
                ("prior_off", _i32p), ("prior_var", _i32p),
                ("point_off", _i32p), ("obs_off", _i32p), ("obs_cam", _i32p), ("obs_pt", _i32p),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double), ("cx", ctypes.c_double),
                ("cy", ctypes.c_double), ("huber_delta", ctypes.c_double)]


class _Options(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("refine", ctypes.c_int32),
                ("lambda_", ctypes.c_double), ("sparse_solve", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("trust_radius", ctypes.c_double), ("refine_last", ctypes.c_int32)]


class _SolveArgs(ctypes.Structure):
    _fields_ = [(n, _vp) for n in ["poses", "points", "edge_meas", "edge_logw", "edge_tau",
                                   "prior_meas", "prior_logw", "obs_uv", "obs_w", "objective",
                                   "status", "factor", "workspace", "edge_logc", "huber_delta"]]


class _BackwardArgs(ctypes.Structure):
    _fields_ = [(n, _vp) for n in ["poses", "points", "edge_meas", "edge_logw", "edge_tau",
                                   "prior_meas", "prior_logw", "obs_uv", "obs_w", "status",
                                   "factor", "seed_pose", "seed_point", "grad_edge_logw",
                                   "grad_edge_tau", "grad_prior_logw", "grad_obs_w", "adjoint",
                                   "workspace"]] + [("mode", ctypes.c_int32), ("dlm_eps", ctypes.c_double),
                                                  ("sweeps", ctypes.c_int32), ("steps", ctypes.c_int32),
                                                  ("edge_logc", _vp), ("grad_edge_logc", _vp),
                                                  ("huber_delta", _vp), ("grad_obs_delta", _vp),
                                                  ("grad_huber_delta", _vp)]


_LIB = None


def lib():
    """The loaded libdnls.so (raises DnlsError if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise DnlsError(f"{LIB_PATH} is missing: build it with paper_2207_09442_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.dnls_plan_create.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(_Problem), ctypes.POINTER(_Options)]
        L.dnls_plan_workspace.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                          ctypes.POINTER(ctypes.c_size_t)]
        L.dnls_plan_flops.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.dnls_plan_schedule.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.dnls_solve.argtypes = [_vp, ctypes.POINTER(_SolveArgs), _vp]
        L.dnls_solve_noalloc.argtypes = [_vp, ctypes.POINTER(_SolveArgs), _vp]
        L.dnls_backward.argtypes = [_vp, ctypes.POINTER(_BackwardArgs), _vp]
        L.dnls_project_grad.argtypes = [ctypes.c_int32, ctypes.c_int64, _vp, _vp, _vp, _vp]
        L.dnls_plan_destroy.argtypes = [_vp]
        L.dnls_last_error.restype = ctypes.c_char_p
        L.dnls_version.restype = ctypes.c_char_p
        for f in ["dnls_plan_create", "dnls_plan_workspace", "dnls_plan_flops", "dnls_plan_schedule", "dnls_solve",
                  "dnls_solve_noalloc", "dnls_backward",
                  "dnls_project_grad", "dnls_plan_destroy"]:
            getattr(L, f).restype = ctypes.c_int
        _LIB = L
    return _LIB


def _check(code: int, what: str):
    if code != 0:
        msg = lib().dnls_last_error().decode()
        raise DnlsError(f"{what} failed with status {code}: {msg}")


def _i32(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    return a, a.ctypes.data_as(_i32p)


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_f64(x, device):
    import torch
    return torch.as_tensor(np.asarray(x) if not isinstance(x, torch.Tensor) else x,
                           dtype=torch.float64, device=device).contiguous()


_LIVE_PLANS = weakref.WeakSet()


@atexit.register
def _close_live_plans():
    """Destroy the plans still alive at interpreter exit while the HIP runtime
    is still up (a destructor run during interpreter finalisation may find it
    torn down)."""
    for p in list(_LIVE_PLANS):
        p.close()


class Plan:
    """A DNLS problem structure with its optimizer settings (dnls_plan_create)
    plus the caller-owned workspace and factor cache (torch device tensors).
    close() (or leaving a `with` block) releases the plan's device tables;
    plans still open at exit are closed by an atexit hook."""

    def __init__(self, problem: dict, iterations: int, lam: float = 0.0, solver: str = "dense",
                 precision: str = "fp64", refine: int = 0, device: str = "cuda", sparse_solve: str = "auto",
                 graph: bool = False, adaptive: bool = False, dogleg: float | None = None,
                 keep_iterates: bool = False, pair: bool = False, refine_last: int = 0):
        """dogleg: initial trust radius of Powell's dogleg, or None;
        keep_iterates: store theta_0 .. theta_{K-1} for the unrolled backward;
        pair: dense solver, two co-resident workgroups per graph when they fit;
        refine_last: mixed precision, refinement sweeps in the last steps only
        (negative: the first steps; 0 = all)."""
        import torch
        self.group = problem["group"]
        self.dof = 6 if self.group == "SE3" else 3
        self.sz = 12 if self.group == "SE3" else 4
        self.K = int(iterations)
        self.device = torch.device(device)
        self.B = len(problem["pose_off"]) - 1
        self.V = int(problem["pose_off"][-1])
        self.E = int(problem["edge_off"][-1])
        self.P = int(problem["prior_off"][-1])
        self.Vp = int(problem["point_off"][-1]) if "point_off" in problem else 0
        self.O = int(problem["obs_off"][-1]) if "obs_off" in problem else 0
        self.obs_off = np.asarray(problem["obs_off"], np.int64) if "obs_off" in problem else None
        keep = []
        pr = _Problem()
        pr.batch = self.B
        pr.group = GROUPS[self.group]
        for name in ["pose_off", "edge_off", "prior_off", "prior_var"]:
            arr, p = _i32(problem[name])
            keep.append(arr)
            setattr(pr, name, p)
        arr, p = _i32(np.asarray(problem["edge_ij"]).reshape(-1))
        keep.append(arr)
        pr.edge_ij = p
        if "point_off" in problem:
            for name in ["point_off", "obs_off", "obs_cam", "obs_pt"]:
                arr, p = _i32(problem[name])
                keep.append(arr)
                setattr(pr, name, p)
            pr.fx, pr.fy, pr.cx, pr.cy = (float(x) for x in problem["intrinsics"])
            pr.huber_delta = float(problem["huber_delta"])
        op = _Options(SOLVERS[solver], PRECISIONS[precision], self.K, int(refine), float(lam),
                      SPARSE_SOLVES[sparse_solve],
                      (FLAG_GRAPH if graph else 0) | (FLAG_ADAPTIVE_LM if adaptive else 0)
                      | (FLAG_DOGLEG if dogleg is not None else 0) | (FLAG_KEEP_ITERATES if keep_iterates else 0)
                      | (FLAG_PAIR if pair else 0),
                      float(dogleg) if dogleg is not None else 0.0, int(refine_last))
        self.config = dict(solver=solver, precision=precision, refine=int(refine), lam=float(lam),
                           sparse_solve=sparse_solve, graph=bool(graph), adaptive=bool(adaptive), dogleg=dogleg,
                           keep_iterates=bool(keep_iterates), pair=bool(pair), refine_last=int(refine_last))
        h = _vp()
        _check(lib().dnls_plan_create(ctypes.byref(h), ctypes.byref(pr), ctypes.byref(op)), "dnls_plan_create")
        self._h = h
        _LIVE_PLANS.add(self)
        # solves run on this plan so far: a backward through the autograd
        # functions must read the factor cache of its own forward
        self.solves = 0
        sw, fb, bw = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().dnls_plan_workspace(h, ctypes.byref(sw), ctypes.byref(fb), ctypes.byref(bw)),
               "dnls_plan_workspace")
        self.solve_ws_bytes, self.factor_bytes, self.backward_ws_bytes = sw.value, fb.value, bw.value
        self.workspace = torch.empty(max(1, sw.value, bw.value) + 256, dtype=torch.uint8, device=self.device)
        self.factor = torch.empty(max(1, fb.value) + 256, dtype=torch.uint8, device=self.device)

    def flops(self):
        """(algorithmic, executed) flops of one numeric factorisation of the
        whole batch (dnls_plan_flops)."""
        a, e = ctypes.c_double(), ctypes.c_double()
        _check(lib().dnls_plan_flops(self._h, ctypes.byref(a), ctypes.byref(e)), "dnls_plan_flops")
        return a.value, e.value

    def schedule(self):
        """The resolved schedule (dnls_plan_schedule): {"pair": bool, "sparse_solve": name}."""
        pair, sp = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().dnls_plan_schedule(self._h, ctypes.byref(pair), ctypes.byref(sp)), "dnls_plan_schedule")
        names = {v: k for k, v in SPARSE_SOLVES.items()}
        return {"pair": bool(pair.value), "sparse_solve": names[sp.value]}

    def pair_active(self):
        return self.schedule()["pair"]

    @staticmethod
    def _aligned(t):
        off = (-t.data_ptr()) % 256
        return ctypes.c_void_p(t.data_ptr() + off)

    def close(self):
        """Destroy the plan's device tables (dnls_plan_destroy); idempotent."""
        h = getattr(self, "_h", None)
        if h is not None and _LIB is not None:
            self._h = None
            _LIB.dnls_plan_destroy(h)
        _LIVE_PLANS.discard(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        # no HIP calls while the interpreter is shutting down: the atexit hook
        # has closed every live plan before that
        if not sys.is_finalizing():
            self.close()

    def _radii(self, huber_delta):
        """Per-problem Huber radii: None, or a float64 tensor on the plan's
        device, 0-dim (one radius shared by every problem, expanded) or [B],
        every radius finite and > 0."""
        import torch
        if huber_delta is None:
            return None
        if not isinstance(huber_delta, torch.Tensor) or huber_delta.dtype != torch.float64 \
                or huber_delta.device != self.device:
            raise DnlsError(f"huber_delta must be a float64 tensor on {self.device}")
        if huber_delta.dim() == 0:
            huber_delta = huber_delta.expand(self.B)
        if tuple(huber_delta.shape) != (self.B,):
            raise DnlsError(f"huber_delta must have shape [B] = [{self.B}] or be 0-dim, "
                            f"got {tuple(huber_delta.shape)}")
        if not bool(torch.isfinite(huber_delta).all()) or not bool((huber_delta > 0).all()):
            raise DnlsError("huber_delta must be finite and > 0")
        return huber_delta.contiguous()

    # ------------------------------------------------------------------
    def solve(self, poses, edge_meas, edge_logw, prior_meas, prior_logw, edge_tau=None, edge_logc=None,
              noalloc=False):
        """Runs K steps in place on `poses` (float64 device tensor [V, 3, 4] or
        [V, 4]); returns (objective [B, K+1], status [B]).  edge_logc: Welsch
        log-radii of the edges [E] (robust loss), or None.  noalloc: through
        dnls_solve_noalloc (the library's scratch in place of the plan's
        workspace)."""
        import torch
        objective = torch.empty(self.B, self.K + 1, dtype=torch.float64, device=self.device)
        status = torch.empty(self.B, dtype=torch.int32, device=self.device)
        a = _SolveArgs()
        a.poses = _ptr(poses)
        a.edge_meas, a.edge_logw, a.edge_tau = _ptr(edge_meas), _ptr(edge_logw), _ptr(edge_tau)
        a.prior_meas, a.prior_logw = _ptr(prior_meas), _ptr(prior_logw)
        a.objective, a.status = _ptr(objective), _ptr(status)
        a.factor = self._aligned(self.factor)
        a.edge_logc = _ptr(edge_logc)
        self._run_solve(a, noalloc)
        return objective, status

    def _run_solve(self, a, noalloc):
        if noalloc:
            a.workspace = None
            _check(lib().dnls_solve_noalloc(self._h, ctypes.byref(a), _stream()), "dnls_solve_noalloc")
        else:
            a.workspace = self._aligned(self.workspace)
            _check(lib().dnls_solve(self._h, ctypes.byref(a), _stream()), "dnls_solve")
        self.solves += 1

    def backward(self, poses, edge_meas, edge_logw, prior_meas, prior_logw, status, seed,
                 edge_tau=None, want_adjoint=False, mode="implicit", eps=1e-3, sweeps=8, steps=None,
                 edge_logc=None):
        """Backward for `seed` = dL/dtheta_K in tangent coordinates [V, dof]:
        mode "implicit" (Proposition 1, with the cached factor), "dlm"
        (direct loss minimisation with perturbation `eps`; no adjoint) or
        "exact" (Proposition 1 with the exact Hessian, `sweeps` refinement
        sweeps preconditioned by the cached factor) or "unroll" (through the
        last `steps` optimizer steps, all K by default; plans made with
        keep_iterates=True; the adjoint is dL/dtheta_{K-steps}); "dlm",
        "exact" and "unroll" on the pose-graph solvers.  With Welsch radii (edge_logc) the
        output also holds their gradient "edge_logc"."""
        import torch
        dev, f64 = self.device, torch.float64
        out = {
            "edge_logw": torch.empty(self.E, dtype=f64, device=dev),
            "edge_tau": torch.empty(self.E, self.dof, dtype=f64, device=dev),
            "prior_logw": torch.empty(self.P, dtype=f64, device=dev),
        }
        if want_adjoint:
            out["adjoint"] = torch.empty(self.V, self.dof, dtype=f64, device=dev)
        if edge_logc is not None:
            out["edge_logc"] = torch.empty(self.E, dtype=f64, device=dev)
        a = _BackwardArgs()
        a.poses = _ptr(poses)
        a.edge_logc, a.grad_edge_logc = _ptr(edge_logc), _ptr(out.get("edge_logc"))
        a.edge_meas, a.edge_logw, a.edge_tau = _ptr(edge_meas), _ptr(edge_logw), _ptr(edge_tau)
        a.prior_meas, a.prior_logw = _ptr(prior_meas), _ptr(prior_logw)
        a.status = _ptr(status)
        a.factor = self._aligned(self.factor)
        a.seed_pose = _ptr(seed.contiguous())
        a.grad_edge_logw, a.grad_edge_tau = _ptr(out["edge_logw"]), _ptr(out["edge_tau"])
        a.grad_prior_logw = _ptr(out["prior_logw"])
        a.adjoint = _ptr(out.get("adjoint"))
        a.workspace = self._aligned(self.workspace)
        a.mode = BACKWARD_MODES[mode]
        a.dlm_eps = float(eps)
        a.sweeps = int(sweeps)
        a.steps = self.K if steps is None else int(steps)
        _check(lib().dnls_backward(self._h, ctypes.byref(a), _stream()), "dnls_backward")
        return out


    # ------------------------------------------------------------------
    def solve_ba(self, cams, points, obs_uv, obs_w, prior_meas, prior_logw, huber_delta=None, noalloc=False):
        """Bundle adjustment (solver "schur"): K steps in place on `cams`
        [Vc, 3, 4] and `points` [Vp, 3]; returns (objective [B, K+1], status [B]).
        huber_delta: per-problem Huber radii [B], or None for the problem's;
        noalloc as for solve."""
        import torch
        objective = torch.empty(self.B, self.K + 1, dtype=torch.float64, device=self.device)
        status = torch.empty(self.B, dtype=torch.int32, device=self.device)
        a = _SolveArgs()
        a.poses, a.points = _ptr(cams), _ptr(points)
        a.obs_uv, a.obs_w = _ptr(obs_uv), _ptr(obs_w)
        a.prior_meas, a.prior_logw = _ptr(prior_meas), _ptr(prior_logw)
        a.objective, a.status = _ptr(objective), _ptr(status)
        a.factor = self._aligned(self.factor)
        hd = self._radii(huber_delta)
        a.huber_delta = _ptr(hd)
        self._run_solve(a, noalloc)
        return objective, status

    def backward_ba(self, cams, points, obs_uv, obs_w, prior_meas, prior_logw, status, seed_cam,
                    seed_pt=None, want_adjoint=False, mode="implicit", eps=1e-3, huber_delta=None):
        """Backward of bundle adjustment: gradients of the observation weights,
        the prior log-weights, the per-observation Huber radii ("obs_delta")
        and the per-problem radii ("huber_delta" [B], their per-problem sums,
        reduced on the device) for tangent seeds on cameras (and points);
        mode "implicit" (Proposition 1) or "dlm" (direct loss minimisation
        with this eps; the adjoint output is not written)."""
        import torch
        dev, f64 = self.device, torch.float64
        out = {"obs_w": torch.empty(self.O, dtype=f64, device=dev),
               "prior_logw": torch.empty(self.P, dtype=f64, device=dev),
               "obs_delta": torch.empty(self.O, dtype=f64, device=dev),
               "huber_delta": torch.empty(self.B, dtype=f64, device=dev)}
        if want_adjoint:
            out["adjoint"] = torch.empty(self.V, 6, dtype=f64, device=dev)
        a = _BackwardArgs()
        a.poses, a.points = _ptr(cams), _ptr(points)
        a.obs_uv, a.obs_w = _ptr(obs_uv), _ptr(obs_w)
        a.prior_meas, a.prior_logw = _ptr(prior_meas), _ptr(prior_logw)
        a.status = _ptr(status)
        a.factor = self._aligned(self.factor)
        a.seed_pose = _ptr(seed_cam.contiguous())
        a.seed_point = _ptr(None if seed_pt is None else seed_pt.contiguous())
        a.grad_obs_w, a.grad_prior_logw = _ptr(out["obs_w"]), _ptr(out["prior_logw"])
        a.grad_obs_delta = _ptr(out["obs_delta"])
        a.grad_huber_delta = _ptr(out["huber_delta"])
        a.adjoint = _ptr(out.get("adjoint"))
        a.workspace = self._aligned(self.workspace)
        a.mode = BACKWARD_MODES[mode]
        a.dlm_eps = float(eps)
        hd = self._radii(huber_delta)
        a.huber_delta = _ptr(hd)
        _check(lib().dnls_backward(self._h, ctypes.byref(a), _stream()), "dnls_backward")
        return out


def project_grad(group: str, poses, grad):
    """Tangent gradient of a Euclidean gradient on the element storage
    (projection operator of Appendix D), computed by the HIP kernel."""
    import torch
    n = poses.shape[0]
    dof = 6 if group == "SE3" else 3
    out = torch.empty(n, dof, dtype=torch.float64, device=poses.device)
    _check(lib().dnls_project_grad(GROUPS[group], n, _ptr(poses.contiguous()), _ptr(grad.contiguous()),
                                   _ptr(out), _stream()), "dnls_project_grad")
    return out


def _same_solve(ctx):
    """The backward reads the plan's factor cache, which the next solve on
    the plan overwrites: refuse a backward whose forward is not the plan's
    latest solve."""
    if ctx.plan.solves != ctx.solve_id:
        raise DnlsError("backward after a later solve on the same Plan: its factor cache now holds the later "
                        "solve's factorisation; use one Plan per forward that is differentiated")


def _autograd_function():
    import torch

    class DNLSFunction(torch.autograd.Function):
        """theta* = argmin S(theta; phi) by K steps, differentiable in
        phi = (edge log-weights, measurement tangent perturbations, prior
        log-weights and, for Welsch edges, their log-radii) by implicit
        differentiation (Proposition 1)."""

        @staticmethod
        def forward(ctx, plan, bwd, poses0, edge_meas, edge_logw, edge_tau, prior_meas, prior_logw, edge_logc=None):
            poses = poses0.detach().clone().contiguous()
            logc = None if edge_logc is None else edge_logc.detach().contiguous()
            objective, status = plan.solve(poses, edge_meas, edge_logw.detach(), prior_meas,
                                           prior_logw.detach(), edge_tau.detach(), edge_logc=logc)
            ctx.plan = plan
            ctx.solve_id = plan.solves
            ctx.bwd = bwd
            ctx.logc = logc
            ctx.save_for_backward(poses, edge_meas, edge_logw, edge_tau, prior_meas, prior_logw, status)
            ctx.mark_non_differentiable(objective, status)
            return poses, objective, status

        @staticmethod
        def backward(ctx, g_poses, g_obj, g_status):
            poses, edge_meas, edge_logw, edge_tau, prior_meas, prior_logw, status = ctx.saved_tensors
            plan = ctx.plan
            if g_poses is None:
                return (None,) * 9
            _same_solve(ctx)
            seed = project_grad(plan.group, poses.reshape(plan.V, -1), g_poses.reshape(plan.V, -1))
            gr = plan.backward(poses, edge_meas, edge_logw.detach(), prior_meas, prior_logw.detach(),
                               status, seed, edge_tau=edge_tau.detach(), edge_logc=ctx.logc, **ctx.bwd)
            return (None, None, None, None, gr["edge_logw"], gr["edge_tau"], None, gr["prior_logw"],
                    gr.get("edge_logc"))

    return DNLSFunction


def _autograd_function_ba():
    import torch

    class DNLSFunctionBA(torch.autograd.Function):
        """Bundle adjustment (cameras*, points*) = argmin S by K steps on the
        Schur solver, differentiable in the observation weights, the prior
        log-weights and (if given) the per-problem Huber radii by implicit
        differentiation (Proposition 1) or DLM."""

        @staticmethod
        def forward(ctx, plan, bwd, cams0, points0, obs_uv, obs_w, prior_meas, prior_logw, huber_delta=None):
            cams = cams0.detach().clone().contiguous()
            points = points0.detach().clone().contiguous()
            hd = None if huber_delta is None else huber_delta.detach().contiguous()
            objective, status = plan.solve_ba(cams, points, obs_uv, obs_w.detach(), prior_meas, prior_logw.detach(),
                                              huber_delta=hd)
            ctx.plan = plan
            ctx.solve_id = plan.solves
            ctx.bwd = bwd
            ctx.hd = hd
            ctx.save_for_backward(cams, points, obs_uv, obs_w, prior_meas, prior_logw, status)
            ctx.mark_non_differentiable(objective, status)
            return cams, points, objective, status

        @staticmethod
        def backward(ctx, g_cams, g_points, g_obj, g_status):
            cams, points, obs_uv, obs_w, prior_meas, prior_logw, status = ctx.saved_tensors
            plan = ctx.plan
            if g_cams is None and g_points is None:
                return (None,) * 9
            _same_solve(ctx)
            if g_cams is None:
                g_cams = torch.zeros_like(cams)
            seed_cam = project_grad("SE3", cams.reshape(plan.V, -1), g_cams.reshape(plan.V, -1))
            seed_pt = None if g_points is None else g_points.contiguous()
            gr = plan.backward_ba(cams, points, obs_uv, obs_w.detach(), prior_meas, prior_logw.detach(), status,
                                  seed_cam, seed_pt, huber_delta=ctx.hd, **ctx.bwd)
            g_delta = None
            if ctx.hd is not None:
                # per-problem radius gradient from the library; a 0-dim radius
                # shared by every problem gets their sum
                g_delta = gr["huber_delta"] if ctx.hd.dim() == 1 else gr["huber_delta"].sum()
            return (None, None, None, None, None, gr["obs_w"], None, gr["prior_logw"], g_delta)

    return DNLSFunctionBA


class _Lazy:
    def __init__(self, make):
        self._make = make
        self._f = None

    def __getattr__(self, k):
        if self._f is None:
            self._f = self._make()
        return getattr(self._f, k)


DNLSFunction = _Lazy(_autograd_function)
DNLSFunctionBA = _Lazy(_autograd_function_ba)


class BALayer:
    """Bundle-adjustment layer: forward(inputs) -> (solution, info) with the
    implicit backward into the observation weights and prior log-weights.
    `inputs` maps cams / points / obs_uv / obs_w / prior_meas / prior_logw to
    float64 device tensors (missing prior log-weights default to zero), and
    optionally huber_delta, per-problem Huber radii [B] (the robust kernel's
    radius, learnable).  backward_mode: "implicit" or "dlm" (with eps)."""

    def __init__(self, plan: Plan, backward_mode: str = "implicit", eps: float = 1e-3):
        if backward_mode not in ("implicit", "dlm"):
            raise DnlsError(f"backward mode {backward_mode!r}: the Schur solver has implicit and dlm")
        self.plan = plan
        self.bwd = dict(mode=backward_mode, eps=eps)

    def forward(self, inputs: dict):
        import torch
        p = self.plan
        prior_logw = inputs.get("prior_logw", torch.zeros(p.P, dtype=torch.float64, device=p.device))
        cams, points, objective, status = DNLSFunctionBA.apply(p, self.bwd, inputs["cams"], inputs["points"],
                                                               inputs["obs_uv"], inputs["obs_w"], inputs["prior_meas"],
                                                               prior_logw, inputs.get("huber_delta"))
        return {"cams": cams, "points": points}, {"objective": objective, "status": status}


class Layer:
    """Theseus-style layer: forward(inputs) -> (solution, info) with the
    implicit backward (Section 3, Listing 1).  `inputs` maps
    poses / edge_meas / edge_logw / edge_tau / prior_meas / prior_logw (and,
    for Welsch-robust edges, edge_logc) to float64 device tensors; missing
    log-weights and tau default to zero, a missing edge_logc means plain
    least squares.  backward_mode: "implicit" (Proposition 1), "dlm",
    "exact" or "unroll" (Section 4.3; the plan needs keep_iterates=True), with
    their options (eps, sweeps, steps) as for Plan.backward."""

    def __init__(self, plan: Plan, backward_mode: str = "implicit", eps: float = 1e-3, sweeps: int = 8,
                 steps: int | None = None):
        if backward_mode not in BACKWARD_MODES:
            raise DnlsError(f"unknown backward mode {backward_mode!r}")
        self.plan = plan
        self.bwd = dict(mode=backward_mode, eps=eps, sweeps=sweeps, steps=steps)

    def forward(self, inputs: dict):
        import torch
        p, dev = self.plan, self.plan.device
        z = lambda *s: torch.zeros(*s, dtype=torch.float64, device=dev)
        edge_logw = inputs.get("edge_logw", z(p.E))
        edge_tau = inputs.get("edge_tau", z(p.E, p.dof))
        prior_logw = inputs.get("prior_logw", z(p.P))
        poses, objective, status = DNLSFunction.apply(p, self.bwd, inputs["poses"], inputs["edge_meas"], edge_logw,
                                                      edge_tau, inputs["prior_meas"], prior_logw,
                                                      inputs.get("edge_logc"))
        return {"poses": poses}, {"objective": objective, "status": status}
