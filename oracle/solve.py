"""The inner loop and the implicit backward, one graph at a time (CPU, float64).

Forward (Section 2 "Solving NLS"; Section 4.2): for t = 0..K-1
  1. linearise every cost at theta_t: c_i, C_i, r_i = w_i c_i, J_i = w_i C_i
     (robust costs reweighted by rho'(s_i), s_i = ||r_i||^2);
  2. H = sum_i J_i^T J_i, g = sum_i J_i^T r_i, S_t = 1/2 sum_i rho(s_i);
  3. damp: H + lambda I (Levenberg-Marquardt with a fixed lambda; lambda = 0 is
     Gauss-Newton);
  4. Cholesky factorisation, delta = (H + lambda I)^-1 g;
  5. retract: X_k <- X_k Exp(-delta_k), Euclidean points p <- p - delta_p.
Then a final linearisation at theta_K (lambda = 0) gives S_K and the
undamped Gauss-Newton Hessian H*, whose factor is kept for the backward.

Adaptive damping (the paper's Levenberg-Marquardt with adaptive damping,
Sections 2 and 3; schedule as read for this implementation): after step 4
the objective is evaluated at the retracted trial point; the step is kept
iff it is strictly smaller than S_t, and then lambda <- lambda / 10,
otherwise theta_t is kept and lambda <- 10 lambda, lambda clamped to
[1e-7, 1e7].

Bundle adjustment eliminates the point blocks with the Schur complement
(Section 4.2, BaSpaCho paragraph): S = B - E C^-1 E^T on the camera block,
then back-substitutes delta_p = C^-1 (g_p - E^T delta_c).

Backward (Section 4.3 "Implicit differentiation", Proposition 1 and its
proof in Appendix H): with v = dL/dtheta at theta_K (tangent, caller-given),
  u = H*^-1 v,   dL/dphi = -d/dphi [ u^T g(theta_K; phi) ]  with u held fixed,
where g = sum_i J_i^T r_i is written as a function of the parameters phi
(log-weights, measurement tangent perturbations Z <- Z Exp(tau), observation
weights) and differentiated by torch.autograd.

Exact-Hessian implicit gradient: the same formula with u = (d^2 S)^-1 v,
d^2 S the Hessian of S(theta_K Exp(delta)) at delta = 0 (torch.autograd),
which closes the gap between the Gauss-Newton reading of Proposition 1 and
the derivative of the re-solved optimum when the residuals are not zero.

Unrolled / truncated gradient: torch.autograd through the last T of the K
plain steps (all K for full unrolling), for the loss whose tangent gradient
at theta_K is v.

Direct loss minimisation (Section 4.3, DLM paragraph; Appendix G): with the
same v, theta_direct minimises S + ||eps theta - v / 2||^2, computed as one
Gauss-Newton step from theta_K in the tangent space there,
  (H* + 2 eps^2 I) delta = -g* + eps v,   theta_direct = theta_K (+) delta,
and dL/dphi ~ (1 / eps) [dS/dphi (theta_K) - dS/dphi (theta_direct)], which
tends to the implicit gradient above as eps -> 0.

Per-graph status: 0 ok, 1 the factorisation failed (not positive definite),
2 a non-finite value appeared.  A failed graph keeps its last iterate, repeats
its last objective value and gets zero gradients.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import costs, lie

DT = torch.float64
OK, NOT_PD, NONFINITE = 0, 1, 2


def _T(x):
    return torch.as_tensor(np.asarray(x), dtype=DT)


# ---------------------------------------------------------------------------
# per-graph views of a batched problem
# ---------------------------------------------------------------------------
@dataclass
class Graph:
    G: lie.Group
    X: torch.Tensor                     # [N, m, m] current poses
    ei: torch.Tensor                    # [E] local index i
    ej: torch.Tensor                    # [E] local index j
    Z: torch.Tensor                     # [E, m, m]
    logw_e: torch.Tensor                # [E]
    pv: torch.Tensor                    # [P] local pose index of each prior
    PZ: torch.Tensor                    # [P, m, m]
    logw_p: torch.Tensor                # [P]
    # bundle adjustment (None for pose graphs)
    pts: torch.Tensor | None = None     # [Np, 3]
    oc: torch.Tensor | None = None      # [O] local camera index
    op: torch.Tensor | None = None      # [O] local point index
    uv: torch.Tensor | None = None      # [O, 2]
    w_o: torch.Tensor | None = None     # [O]
    intr: tuple | None = None
    delta: float = 0.0
    tau: torch.Tensor | None = None     # [E, dof] measurement tangent perturbation
    logc_e: torch.Tensor | None = None  # [E] Welsch log-radius of each edge (None: plain least squares)

    @property
    def n_pose(self):
        return self.X.shape[0]

    @property
    def is_ba(self):
        return self.pts is not None


def graphs_of(problem: dict, poses=None, points=None) -> list[Graph]:
    G = lie.group(problem["group"])
    poses = problem["poses_init"] if poses is None else poses
    out = []
    B = len(problem["pose_off"]) - 1
    for b in range(B):
        p0, p1 = int(problem["pose_off"][b]), int(problem["pose_off"][b + 1])
        e0, e1 = int(problem["edge_off"][b]), int(problem["edge_off"][b + 1])
        q0, q1 = int(problem["prior_off"][b]), int(problem["prior_off"][b + 1])
        ij = np.asarray(problem["edge_ij"][e0:e1], dtype=np.int64).reshape(-1, 2) - p0
        g = Graph(
            G=G,
            X=G.from_storage(_T(poses[p0:p1])),
            ei=torch.as_tensor(ij[:, 0]), ej=torch.as_tensor(ij[:, 1]),
            Z=G.from_storage(_T(problem["edge_meas"][e0:e1]).reshape(-1, *np.shape(poses)[1:])),
            logw_e=_T(problem["edge_logw"][e0:e1]),
            pv=torch.as_tensor(np.asarray(problem["prior_var"][q0:q1], dtype=np.int64) - p0),
            PZ=G.from_storage(_T(problem["prior_meas"][q0:q1])),
            logw_p=_T(problem["prior_logw"][q0:q1]),
        )
        if problem.get("edge_logc") is not None:
            g.logc_e = _T(problem["edge_logc"][e0:e1])
        if "point_off" in problem:
            t0, t1 = int(problem["point_off"][b]), int(problem["point_off"][b + 1])
            o0, o1 = int(problem["obs_off"][b]), int(problem["obs_off"][b + 1])
            pts = problem["points_init"] if points is None else points
            g.pts = _T(pts[t0:t1])
            g.oc = torch.as_tensor(np.asarray(problem["obs_cam"][o0:o1], dtype=np.int64) - p0)
            g.op = torch.as_tensor(np.asarray(problem["obs_pt"][o0:o1], dtype=np.int64) - t0)
            g.uv = _T(problem["obs_uv"][o0:o1])
            g.w_o = _T(problem["obs_w"][o0:o1])
            g.intr = tuple(float(x) for x in problem["intrinsics"])
            g.delta = float(problem["huber_delta"])
        out.append(g)
    return out


# ---------------------------------------------------------------------------
# linearisation
# ---------------------------------------------------------------------------
@dataclass
class Lin:
    S: torch.Tensor                      # objective 1/2 sum rho(s)
    H: torch.Tensor                      # pose-graph: [n, n]; BA: camera block [6Nc, 6Nc]
    g: torch.Tensor                      # pose-graph: [n];    BA: camera part [6Nc]
    # bundle adjustment only
    E: torch.Tensor | None = None        # [6Nc, 3Np]
    C: torch.Tensor | None = None        # [Np, 3, 3]
    gp: torch.Tensor | None = None       # [Np, 3]
    extra: dict = field(default_factory=dict)


def _scatter_blocks(N: int, d: int, rows, cols, blocks) -> torch.Tensor:
    """Sum d x d blocks into a dense [N*d, N*d] matrix."""
    Hb = torch.zeros(N, N, d, d, dtype=DT)
    Hb = Hb.index_put((rows, cols), blocks, accumulate=True)
    return Hb.permute(0, 2, 1, 3).reshape(N * d, N * d)


def _scatter_vec(N: int, d: int, idx, vecs) -> torch.Tensor:
    return torch.zeros(N, d, dtype=DT).index_add(0, idx, vecs).reshape(N * d)


def pose_costs(g: Graph, X: torch.Tensor, tau=None, logw_e=None, logw_p=None):
    """Residual/Jacobian blocks of the relative-pose and prior costs."""
    G = g.G
    Z = g.Z if tau is None else g.Z @ G.exp(tau)
    logw_e = g.logw_e if logw_e is None else logw_e
    logw_p = g.logw_p if logw_p is None else logw_p
    c_e, Ci, Cj = costs.between(G, X[g.ei], X[g.ej], Z)
    c_p, Cp = costs.prior(G, X[g.pv], g.PZ)
    return dict(c_e=c_e, Ci=Ci, Cj=Cj, w_e=torch.exp(logw_e), c_p=c_p, Cp=Cp, w_p=torch.exp(logw_p))


def welsch(s: torch.Tensor, logc: torch.Tensor):
    """Welsch robust loss on the squared weighted residual s with radius
    c = exp(logc): rho(s) = c^2 (1 - exp(-s / c^2)) and rho'(s) = exp(-s / c^2)."""
    c2 = torch.exp(2.0 * logc)
    return c2 * (1.0 - torch.exp(-s / c2)), torch.exp(-s / c2)


def linearize_pose_graph(g: Graph, X: torch.Tensor, tau=None, logw_e=None, logw_p=None, logc_e=None) -> Lin:
    """Normal equations of the pose-graph objective.  With Welsch radii on the
    edges (g.logc_e, or logc_e) the edges enter by first-order reweighting:
    J and r scaled by sqrt(rho'(s)), s = ||w c||^2, and S = 1/2 sum rho(s)."""
    G, d, N = g.G, g.G.dof, X.shape[0]
    k = pose_costs(g, X, tau, logw_e, logw_p)
    logc_e = g.logc_e if logc_e is None else logc_e
    se = (k["w_e"] ** 2) * (k["c_e"] ** 2).sum(-1)
    if logc_e is not None:
        # reweighted squared weight w^2 rho'(s), without a square root in the
        # autograd graph (rho' underflows to 0 on gross outliers)
        rho_e, drho_e = welsch(se, logc_e)
        w2e = (k["w_e"] ** 2 * drho_e)[:, None, None]
    else:
        rho_e = se
        w2e = (k["w_e"] ** 2)[:, None, None]
    w2p = (k["w_p"] ** 2)[:, None, None]
    Ci, Cj, Cp = k["Ci"], k["Cj"], k["Cp"]
    tr = lambda A: A.transpose(-1, -2)
    rows = torch.cat([g.ei, g.ej, g.ei, g.ej, g.pv])
    cols = torch.cat([g.ei, g.ej, g.ej, g.ei, g.pv])
    blocks = torch.cat([w2e * tr(Ci) @ Ci, w2e * tr(Cj) @ Cj, w2e * tr(Ci) @ Cj,
                        w2e * tr(Cj) @ Ci, w2p * tr(Cp) @ Cp])
    H = _scatter_blocks(N, d, rows, cols, blocks)
    ge_i = (w2e * tr(Ci) @ k["c_e"][..., None])[..., 0]
    ge_j = (w2e * tr(Cj) @ k["c_e"][..., None])[..., 0]
    gp = (w2p * tr(Cp) @ k["c_p"][..., None])[..., 0]
    gvec = _scatter_vec(N, d, torch.cat([g.ei, g.ej, g.pv]), torch.cat([ge_i, ge_j, gp]))
    S = 0.5 * rho_e.sum() + 0.5 * ((k["w_p"] ** 2) * (k["c_p"] ** 2).sum(-1)).sum()
    return Lin(S=S, H=H, g=gvec, extra=k)


def objective_and_gradient_pose_graph(g: Graph, X: torch.Tensor, tau=None, logw_e=None, logw_p=None):
    """S and g = sum_i J_i^T r_i of the (non-robust) pose-graph objective
    without forming H: what the backward differentiates on graphs too large
    for a dense matrix.  Returns (S, g [n], cost blocks)."""
    d, N = g.G.dof, X.shape[0]
    k = pose_costs(g, X, tau, logw_e, logw_p)
    w2e = (k["w_e"] ** 2)[:, None, None]
    w2p = (k["w_p"] ** 2)[:, None, None]
    tr = lambda A: A.transpose(-1, -2)
    ge_i = (w2e * tr(k["Ci"]) @ k["c_e"][..., None])[..., 0]
    ge_j = (w2e * tr(k["Cj"]) @ k["c_e"][..., None])[..., 0]
    gp = (w2p * tr(k["Cp"]) @ k["c_p"][..., None])[..., 0]
    gvec = _scatter_vec(N, d, torch.cat([g.ei, g.ej, g.pv]), torch.cat([ge_i, ge_j, gp]))
    S = 0.5 * ((k["w_e"] ** 2) * (k["c_e"] ** 2).sum(-1)).sum() + \
        0.5 * ((k["w_p"] ** 2) * (k["c_p"] ** 2).sum(-1)).sum()
    return S, gvec, k


def linearize_pose_graph_sparse(g: Graph, X: torch.Tensor, tau=None):
    """Same normal equations as linearize_pose_graph, as a scipy CSR matrix
    (for graphs too large for a dense matrix); returns (S, H, g)."""
    import scipy.sparse as sp
    d, N = g.G.dof, X.shape[0]
    S, gvec, k = objective_and_gradient_pose_graph(g, X, tau)
    w2e = (k["w_e"] ** 2)[:, None, None]
    w2p = (k["w_p"] ** 2)[:, None, None]
    Ci, Cj, Cp = k["Ci"], k["Cj"], k["Cp"]
    tr = lambda A: A.transpose(-1, -2)
    rows = torch.cat([g.ei, g.ej, g.ei, g.ej, g.pv]).numpy()
    cols = torch.cat([g.ei, g.ej, g.ej, g.ei, g.pv]).numpy()
    blocks = torch.cat([w2e * tr(Ci) @ Ci, w2e * tr(Cj) @ Cj, w2e * tr(Ci) @ Cj,
                        w2e * tr(Cj) @ Ci, w2p * tr(Cp) @ Cp]).numpy()
    rr = (rows[:, None, None] * d + np.arange(d)[None, :, None]) + 0 * np.arange(d)[None, None, :]
    cc = (cols[:, None, None] * d + np.arange(d)[None, None, :]) + 0 * np.arange(d)[None, :, None]
    H = sp.coo_matrix((blocks.ravel(), (rr.ravel(), cc.ravel())), shape=(N * d, N * d)).tocsr()
    return float(S), H, gvec.numpy()


def ba_costs(g: Graph, X: torch.Tensor, pts: torch.Tensor, w_o=None, logw_p=None, delta_o=None):
    """Observation and prior costs of a BA problem; delta_o, a per-observation
    Huber radius, defaults to the problem's radius."""
    w_o = g.w_o if w_o is None else w_o
    logw_p = g.logw_p if logw_p is None else logw_p
    c, Cc, Cq = costs.reprojection(X[g.oc], pts[g.op], g.uv, g.intr)
    r2 = (w_o ** 2) * (c ** 2).sum(-1)
    rho, drho = costs.huber(r2, g.delta if delta_o is None else delta_o)
    c_p, Cp = costs.prior(g.G, X[g.pv], g.PZ)
    return dict(c=c, Cc=Cc, Cq=Cq, w_o=w_o, rho=rho, drho=drho, c_p=c_p, Cp=Cp,
                w_p=torch.exp(logw_p))


def ba_objective(g: Graph, X: torch.Tensor, pts: torch.Tensor, w_o=None, logw_p=None, delta_o=None) -> torch.Tensor:
    """S = 1/2 sum_o rho(w_o^2 ||c_o||^2) + 1/2 sum_p w_p^2 ||c_p||^2 (Huber rho
    on the observations, as in linearize_ba)."""
    k = ba_costs(g, X, pts, w_o, logw_p, delta_o)
    return 0.5 * k["rho"].sum() + 0.5 * ((k["w_p"] ** 2) * (k["c_p"] ** 2).sum(-1)).sum()


def linearize_ba(g: Graph, X: torch.Tensor, pts: torch.Tensor, w_o=None, logw_p=None, delta_o=None) -> Lin:
    Nc, Np = X.shape[0], pts.shape[0]
    k = ba_costs(g, X, pts, w_o, logw_p, delta_o)
    tr = lambda A: A.transpose(-1, -2)
    a = (k["drho"] * k["w_o"] ** 2)[:, None, None]          # rho' w^2
    Cc, Cq = k["Cc"], k["Cq"]
    w2p = (k["w_p"] ** 2)[:, None, None]
    B = _scatter_blocks(Nc, 6, torch.cat([g.oc, g.pv]), torch.cat([g.oc, g.pv]),
                        torch.cat([a * tr(Cc) @ Cc, w2p * tr(k["Cp"]) @ k["Cp"]]))
    Eb = torch.zeros(Nc, Np, 6, 3, dtype=DT).index_put((g.oc, g.op), a * tr(Cc) @ Cq, accumulate=True)
    E = Eb.permute(0, 2, 1, 3).reshape(Nc * 6, Np * 3)
    C = torch.zeros(Np, 3, 3, dtype=DT).index_add(0, g.op, a * tr(Cq) @ Cq)
    gc = _scatter_vec(Nc, 6, torch.cat([g.oc, g.pv]),
                      torch.cat([(a * tr(Cc) @ k["c"][..., None])[..., 0],
                                 (w2p * tr(k["Cp"]) @ k["c_p"][..., None])[..., 0]]))
    gp = torch.zeros(Np, 3, dtype=DT).index_add(0, g.op, (a * tr(Cq) @ k["c"][..., None])[..., 0])
    S = 0.5 * k["rho"].sum() + 0.5 * ((k["w_p"] ** 2) * (k["c_p"] ** 2).sum(-1)).sum()
    return Lin(S=S, H=B, g=gc, E=E, C=C, gp=gp, extra=k)


# ---------------------------------------------------------------------------
# linear solves
# ---------------------------------------------------------------------------
def _chol(A: torch.Tensor):
    L, info = torch.linalg.cholesky_ex(A)
    return (L if int(info) == 0 else None)


def _finite(*ts) -> bool:
    return all(bool(torch.isfinite(t).all()) for t in ts)


def pose_graph_step(lin: Lin, lam: float):
    """delta = (H + lam I)^-1 g by Cholesky; returns (delta, L) or (None, None)."""
    n = lin.H.shape[0]
    L = _chol(lin.H + lam * torch.eye(n, dtype=DT))
    if L is None:
        return None, None
    return torch.cholesky_solve(lin.g[:, None], L)[:, 0], L


def schur_factor(lin: Lin, lam: float):
    """Damped Schur complement on the camera block and its Cholesky factor."""
    nc = lin.H.shape[0]
    Cl = lin.C + lam * torch.eye(3, dtype=DT)
    Ci = torch.linalg.inv(Cl)                                   # [Np, 3, 3]
    Np = Ci.shape[0]
    # E C^-1 with C^-1 block-diagonal: multiply each point's 3 columns by its block
    EC = torch.einsum("rpk,pkj->rpj", lin.E.reshape(nc, Np, 3), Ci).reshape(nc, 3 * Np)
    Sm = lin.H + lam * torch.eye(nc, dtype=DT) - EC @ lin.E.T
    L = _chol(Sm)
    return L, Ci, EC


def schur_solve(lin: Lin, L, Ci, EC, rhs_c, rhs_p):
    """Solve [[B, E], [E^T, C]] [x_c; x_p] = [rhs_c; rhs_p] given the Schur factor."""
    rc = rhs_c - EC @ rhs_p.reshape(-1)
    xc = torch.cholesky_solve(rc[:, None], L)[:, 0]
    xp = (Ci @ (rhs_p - (lin.E.T @ xc).reshape(-1, 3))[..., None])[..., 0]
    return xc, xp


# ---------------------------------------------------------------------------
# forward
# ---------------------------------------------------------------------------
@dataclass
class GraphResult:
    X: torch.Tensor
    pts: torch.Tensor | None
    objective: list
    status: int
    lin: Lin | None = None        # final linearisation at theta_K
    factor: tuple | None = None   # cached factor of H* (or of the Schur complement)
    lambdas: list | None = None   # adaptive damping: lambda used at each step
    radii: list | None = None     # dogleg: trust radius used at each step


LAMBDA_MIN, LAMBDA_MAX = 1e-7, 1e7


RADIUS_MAX = 1e4


def dogleg_step(lin: Lin, L, delta_gn, lam: float, radius: float):
    """Powell's dogleg inside the trust region ||delta|| <= radius for the
    model m(delta) = S - g^T delta + 1/2 delta^T (H + lam I) delta of the step
    theta (-) delta: the Gauss-Newton point if it lies inside, else the
    scaled gradient if even the Cauchy point lies outside, else the point of
    the dogleg path on the boundary.  Returns (delta, on_boundary, predicted
    decrease m(0) - m(delta))."""
    n = lin.H.shape[0]
    Hl = lin.H + lam * torch.eye(n, dtype=DT)
    g = lin.g
    if float(delta_gn.norm()) <= radius:
        delta, boundary = delta_gn, False
    else:
        gg = float(g @ g)
        alpha = gg / float(g @ (Hl @ g))
        if alpha * gg ** 0.5 >= radius:
            delta = (radius / gg ** 0.5) * g
        else:
            sd = alpha * g
            dd = delta_gn - sd
            a, b, c = float(dd @ dd), 2.0 * float(sd @ dd), alpha * alpha * gg - radius * radius
            beta = (-b + (b * b - 4.0 * a * c) ** 0.5) / (2.0 * a)
            delta = sd + beta * dd
        boundary = True
    pred = float(g @ delta) - 0.5 * float(delta @ (Hl @ delta))
    return delta, boundary, pred


def solve_graph(g: Graph, iterations: int, lam: float, tau=None, adaptive: bool = False,
                dogleg_radius: float | None = None) -> GraphResult:
    """K optimizer steps on one graph then the final linearisation.  Fixed
    damping by default; adaptive=True adapts lambda per step; dogleg_radius
    runs Powell's dogleg with that initial trust radius (accept iff the
    objective strictly decreases; with rho = actual / predicted decrease the
    radius becomes ||delta|| / 4 if rho < 1/4 and min(2 radius, 1e4) if
    rho > 3/4 on the boundary)."""
    if tau is None:
        tau = g.tau
    X = g.X.clone()
    pts = None if g.pts is None else g.pts.clone()
    obj, status = [], OK
    lambdas = [] if adaptive else None
    radius = dogleg_radius
    radii = [] if dogleg_radius is not None else None
    for _ in range(iterations):
        if g.is_ba:
            lin = linearize_ba(g, X, pts)
            ok = _finite(lin.S, lin.H, lin.g, lin.E, lin.C, lin.gp)
        else:
            lin = linearize_pose_graph(g, X, tau=tau)
            ok = _finite(lin.S, lin.H, lin.g)
        obj.append(float(lin.S))
        if not ok:
            status = NONFINITE
            break
        if g.is_ba:
            L, Ci, EC = schur_factor(lin, lam)
            if L is None:
                status = NOT_PD
                break
            dc, dp = schur_solve(lin, L, Ci, EC, lin.g, lin.gp)
            if radius is not None:
                # the dogleg over cameras and points together (full system)
                radii.append(radius)
                nc = lin.H.shape[0]
                full = Lin(S=lin.S, H=ba_full_system(lin), g=torch.cat([lin.g, lin.gp.reshape(-1)]))
                delta, boundary, pred = dogleg_step(full, None, torch.cat([dc, dp.reshape(-1)]), lam, radius)
                X_trial = g.G.retract(X, -delta[:nc].reshape(-1, 6))
                pts_trial = pts - delta[nc:].reshape(-1, 3)
                s_trial = float(ba_objective(g, X_trial, pts_trial))
                rho = (float(lin.S) - s_trial) / pred
                if s_trial < float(lin.S):
                    X, pts = X_trial, pts_trial
                if not rho >= 0.25:
                    radius = 0.25 * float(delta.norm())
                elif rho > 0.75 and boundary:
                    radius = min(2.0 * radius, RADIUS_MAX)
                continue
            X_trial = g.G.retract(X, -dc.reshape(-1, 6))
            pts_trial = pts - dp
            if adaptive:
                # the same rule as for pose graphs, on cameras and points together
                lambdas.append(lam)
                s_trial = float(ba_objective(g, X_trial, pts_trial))
                if s_trial < float(lin.S):
                    X, pts, lam = X_trial, pts_trial, max(lam / 10.0, LAMBDA_MIN)
                else:
                    lam = min(lam * 10.0, LAMBDA_MAX)
            else:
                X, pts = X_trial, pts_trial
        else:
            delta, L = pose_graph_step(lin, lam)
            if delta is None:
                status = NOT_PD
                break
            if radius is not None:
                radii.append(radius)
                delta, boundary, pred = dogleg_step(lin, L, delta, lam, radius)
                trial = g.G.retract(X, -delta.reshape(-1, g.G.dof))
                s_trial = float(linearize_pose_graph(g, trial, tau=tau).S)
                rho = (float(lin.S) - s_trial) / pred
                if s_trial < float(lin.S):
                    X = trial
                if not rho >= 0.25:                    # NaN shrinks too
                    radius = 0.25 * float(delta.norm())
                elif rho > 0.75 and boundary:
                    radius = min(2.0 * radius, RADIUS_MAX)
                continue
            trial = g.G.retract(X, -delta.reshape(-1, g.G.dof))
            if adaptive:
                lambdas.append(lam)
                s_trial = float(linearize_pose_graph(g, trial, tau=tau).S)
                if s_trial < float(lin.S):          # NaN compares false: rejected
                    X, lam = trial, max(lam / 10.0, LAMBDA_MIN)
                else:
                    lam = min(lam * 10.0, LAMBDA_MAX)
            else:
                X = trial
    res = GraphResult(X=X, pts=pts, objective=obj, status=status, lambdas=lambdas, radii=radii)
    if status != OK:
        res.objective = obj + [obj[-1]] * (iterations + 1 - len(obj))
        return res
    # final linearisation at theta_K, undamped
    lin = linearize_ba(g, X, pts) if g.is_ba else linearize_pose_graph(g, X, tau=tau)
    res.objective = obj + [float(lin.S)]
    res.lin = lin
    if not _finite(lin.S, lin.H, lin.g):
        res.status = NONFINITE
        return res
    if g.is_ba:
        L, Ci, EC = schur_factor(lin, 0.0)
        res.factor = None if L is None else (L, Ci, EC)
    else:
        L = _chol(lin.H)
        res.factor = None if L is None else (L,)
    if res.factor is None:
        res.status = NOT_PD
    return res


def solve(problem: dict, iterations: int, lam: float = 0.0, graphs=None):
    """Run the inner loop on every graph; returns (results, stacked outputs)."""
    gs = graphs_of(problem) if graphs is None else graphs
    results = [solve_graph(g, iterations, lam) for g in gs]
    G = lie.group(problem["group"])
    poses = torch.cat([G.to_storage(r.X) for r in results]).numpy()
    out = dict(poses=poses, objective=np.array([r.objective for r in results]),
               status=np.array([r.status for r in results], dtype=np.int32))
    if gs and gs[0].is_ba:
        out["points"] = torch.cat([r.pts for r in results]).numpy()
    return results, out


# ---------------------------------------------------------------------------
# backward (Proposition 1)
# ---------------------------------------------------------------------------
def adjoint(res: GraphResult, v_pose: torch.Tensor, v_pts=None):
    """u = H*^-1 v with the factor kept by the final linearisation."""
    if res.lin.E is None:
        (L,) = res.factor
        return torch.cholesky_solve(v_pose.reshape(-1, 1), L)[:, 0].reshape(v_pose.shape), None
    L, Ci, EC = res.factor
    uc, up = schur_solve(res.lin, L, Ci, EC, v_pose.reshape(-1), v_pts)
    return uc.reshape(v_pose.shape), up


def implicit_grad_graph(g: Graph, res: GraphResult, v_pose, v_pts=None) -> dict:
    """dL/dphi = -d/dphi [u^T g(theta_K; phi)] for the graph's parameters."""
    d = g.G.dof
    if res.status != OK:
        z = dict(edge_logw=torch.zeros(len(g.ei), dtype=DT), prior_logw=torch.zeros(len(g.pv), dtype=DT),
                 tau=torch.zeros(len(g.ei), d, dtype=DT))
        if g.is_ba:
            z = dict(obs_w=torch.zeros(len(g.oc), dtype=DT), prior_logw=torch.zeros(len(g.pv), dtype=DT),
                     obs_delta=torch.zeros(len(g.oc), dtype=DT))
        return z
    u, up = adjoint(res, v_pose, v_pts)
    if g.is_ba:
        w = g.w_o.clone().requires_grad_(True)
        lp = g.logw_p.clone().requires_grad_(True)
        dl = torch.full((len(g.oc),), float(g.delta), dtype=DT).requires_grad_(True)
        lin = linearize_ba(g, res.X, res.pts, w_o=w, logw_p=lp, delta_o=dl)
        Y = (lin.g * u.reshape(-1)).sum() + (lin.gp * up).sum()
        dw, dp, dd = torch.autograd.grad(Y, [w, lp, dl])
        return dict(obs_w=-dw, prior_logw=-dp, obs_delta=-dd, u=u, u_pts=up)
    le = g.logw_e.clone().requires_grad_(True)
    lp = g.logw_p.clone().requires_grad_(True)
    tau0 = g.tau if g.tau is not None else torch.zeros(len(g.ei), d, dtype=DT)
    tau = tau0.clone().requires_grad_(True)
    params = [le, lp, tau]
    lc = None
    if g.logc_e is not None:
        lc = g.logc_e.clone().requires_grad_(True)
        params.append(lc)
    lin = linearize_pose_graph(g, res.X, tau=tau, logw_e=le, logw_p=lp, logc_e=lc)
    Y = (lin.g * u.reshape(-1)).sum()
    grads = torch.autograd.grad(Y, params)
    out = dict(edge_logw=-grads[0], prior_logw=-grads[1], tau=-grads[2], u=u)
    if lc is not None:
        out["edge_logc"] = -grads[3]
    return out


def exact_hessian_graph(g: Graph, X: torch.Tensor) -> torch.Tensor:
    """Hessian of f(delta) = S(X Exp(delta)) at delta = 0 (right
    perturbations of every pose, the tangent chart the optimizer steps in):
    the Gauss-Newton Hessian plus the second-order residual terms."""
    n = X.shape[0] * g.G.dof
    tau = g.tau if g.tau is not None else None

    def f(delta):
        return linearize_pose_graph(g, g.G.retract(X, delta.reshape(X.shape[0], -1)), tau=tau).S

    return torch.autograd.functional.hessian(f, torch.zeros(n, dtype=DT))


def exact_implicit_grad_graph(g: Graph, res: GraphResult, v_pose) -> dict:
    """Proposition 1 with the exact Hessian in place of the Gauss-Newton one:
    u = (d^2 S)^-1 v, then dL/dphi = -d/dphi [u^T g(theta_K; phi)] as in the
    implicit gradient.  At a stationary point this is the derivative of the
    re-solved optimum (the implicit function theorem applied to g = 0)."""
    d = g.G.dof
    if res.status != OK:
        return dict(edge_logw=torch.zeros(len(g.ei), dtype=DT), prior_logw=torch.zeros(len(g.pv), dtype=DT),
                    tau=torch.zeros(len(g.ei), d, dtype=DT), u=torch.zeros(res.X.shape[0], d, dtype=DT))
    Hx = exact_hessian_graph(g, res.X)
    u = torch.linalg.solve(Hx, torch.as_tensor(v_pose, dtype=DT).reshape(-1)).reshape(-1, d)
    le = g.logw_e.clone().requires_grad_(True)
    lp = g.logw_p.clone().requires_grad_(True)
    tau0 = g.tau if g.tau is not None else torch.zeros(len(g.ei), d, dtype=DT)
    tau = tau0.clone().requires_grad_(True)
    lin = linearize_pose_graph(g, res.X, tau=tau, logw_e=le, logw_p=lp)
    Y = (lin.g * u.reshape(-1)).sum()
    de, dp, dt = torch.autograd.grad(Y, [le, lp, tau])
    return dict(edge_logw=-de, prior_logw=-dp, tau=-dt, u=u)


def unrolled_grad_graph(g: Graph, iterations: int, lam: float, v_pose, steps: int | None = None) -> dict:
    """Gradient by differentiating through the optimizer's own steps
    (Section 4.3, unrolling; truncated unrolling keeps only the last `steps`
    of the K steps): torch.autograd through the plain (fixed-damping) step
    delta = (H + lam I)^-1 g, X <- X Exp(-delta), of the log-weights, prior
    log-weights and measurement tangents, for the loss whose tangent gradient
    at theta_K is v: L = sum_p v_p . Log(theta_K,p^-1 X_p) with theta_K held
    fixed.  Also returns dL/dxi at theta_{K - steps} ("adjoint")."""
    import dataclasses
    d = g.G.dof
    T = iterations if steps is None else steps
    start = solve_graph(g, iterations - T, lam) if T < iterations else None
    X0 = g.X if start is None else start.X.detach()
    le = g.logw_e.clone().requires_grad_(True)
    lp = g.logw_p.clone().requires_grad_(True)
    tau0 = g.tau if g.tau is not None else torch.zeros(len(g.ei), d, dtype=DT)
    tau = tau0.clone().requires_grad_(True)
    xi = torch.zeros(X0.shape[0], d, dtype=DT, requires_grad=True)
    gg = dataclasses.replace(g, X=g.G.retract(X0, xi), logw_e=le, logw_p=lp, tau=tau)
    r = solve_graph(gg, T, lam)
    XK = r.X.detach()
    L = (g.G.log(g.G.inv(XK) @ r.X) * torch.as_tensor(v_pose, dtype=DT)).sum()
    de, dp, dt, dx = torch.autograd.grad(L, [le, lp, tau, xi], allow_unused=True)
    z = lambda t, like: torch.zeros_like(like) if t is None else t
    return dict(edge_logw=z(de, le), prior_logw=z(dp, lp), tau=z(dt, tau), adjoint=z(dx, xi), status=r.status)


def dlm_grad_graph(g: Graph, res: GraphResult, v_pose, eps: float) -> dict:
    """Direct-loss-minimisation gradient of a pose graph (see the module
    docstring): the objective's parameter gradient at theta_K and at
    theta_direct, differenced and divided by eps."""
    d = g.G.dof
    if res.status != OK:
        return dict(edge_logw=torch.zeros(len(g.ei), dtype=DT), prior_logw=torch.zeros(len(g.pv), dtype=DT),
                    tau=torch.zeros(len(g.ei), d, dtype=DT))
    tau0 = g.tau if g.tau is not None else torch.zeros(len(g.ei), d, dtype=DT)

    def dS(X):
        le = g.logw_e.clone().requires_grad_(True)
        lp = g.logw_p.clone().requires_grad_(True)
        tau = tau0.clone().requires_grad_(True)
        params = [le, lp, tau]
        lc = None
        if g.logc_e is not None:
            lc = g.logc_e.clone().requires_grad_(True)
            params.append(lc)
        lin = linearize_pose_graph(g, X, tau=tau, logw_e=le, logw_p=lp, logc_e=lc)
        return torch.autograd.grad(lin.S, params)

    lin = res.lin
    n = lin.H.shape[0]
    rhs = -lin.g + eps * torch.as_tensor(v_pose, dtype=DT).reshape(-1)
    delta = torch.linalg.solve(lin.H + 2.0 * eps * eps * torch.eye(n, dtype=DT), rhs)
    X_direct = g.G.retract(res.X, delta.reshape(-1, d))
    a, b = dS(res.X), dS(X_direct)
    out = dict(edge_logw=(a[0] - b[0]) / eps, prior_logw=(a[1] - b[1]) / eps, tau=(a[2] - b[2]) / eps,
               delta=delta.reshape(-1, d))
    if g.logc_e is not None:
        out["edge_logc"] = (a[3] - b[3]) / eps
    return out


def ba_full_system(lin: Lin) -> torch.Tensor:
    """The bundle-adjustment normal matrix over cameras and points together,
    [[H, E], [E^T, blockdiag(C)]], from a linearisation."""
    nc, npt = lin.H.shape[0], lin.C.shape[0]
    Hf = torch.zeros(nc + 3 * npt, nc + 3 * npt, dtype=DT)
    Hf[:nc, :nc] = lin.H
    Hf[:nc, nc:] = lin.E
    Hf[nc:, :nc] = lin.E.T
    Hf[nc:, nc:] = torch.block_diag(*lin.C)
    return Hf


def dlm_grad_ba(g: Graph, res: GraphResult, v_pose, v_pts, eps: float) -> dict:
    """Direct-loss-minimisation gradient of a bundle-adjustment problem
    (Section 4.3, Appendix G) for the observation weights and the prior
    log-weights: one Gauss-Newton step on S + ||eps theta - v/2||^2 over
    cameras and points together, (H* + 2 eps^2 I) delta = -g* + eps v on the
    full system, theta_direct = (X Exp(delta_c), p + delta_p), then the
    objective's parameter gradients differenced and divided by eps."""
    if res.status != OK:
        return dict(obs_w=torch.zeros(len(g.oc), dtype=DT), prior_logw=torch.zeros(len(g.pv), dtype=DT),
                    obs_delta=torch.zeros(len(g.oc), dtype=DT))
    lin = res.lin
    nc = lin.H.shape[0]
    v = torch.cat([torch.as_tensor(v_pose, dtype=DT).reshape(-1),
                   (torch.zeros(lin.gp.numel(), dtype=DT) if v_pts is None
                    else torch.as_tensor(v_pts, dtype=DT).reshape(-1))])
    Hf = ba_full_system(lin)
    rhs = -torch.cat([lin.g, lin.gp.reshape(-1)]) + eps * v
    delta = torch.linalg.solve(Hf + 2.0 * eps * eps * torch.eye(Hf.shape[0], dtype=DT), rhs)
    X_d = g.G.retract(res.X, delta[:nc].reshape(-1, 6))
    p_d = res.pts + delta[nc:].reshape(-1, 3)

    def dS(X, pts):
        w = g.w_o.clone().requires_grad_(True)
        lp = g.logw_p.clone().requires_grad_(True)
        dl = torch.full((len(g.oc),), float(g.delta), dtype=DT).requires_grad_(True)
        return torch.autograd.grad(ba_objective(g, X, pts, w_o=w, logw_p=lp, delta_o=dl), [w, lp, dl])

    a, b = dS(res.X, res.pts), dS(X_d, p_d)
    return dict(obs_w=(a[0] - b[0]) / eps, prior_logw=(a[1] - b[1]) / eps, obs_delta=(a[2] - b[2]) / eps,
                delta=delta)


def backward(problem: dict, results: list, v_pose: np.ndarray, v_pts=None, graphs=None) -> dict:
    gs = graphs_of(problem) if graphs is None else graphs
    outs = []
    for b, (g, r) in enumerate(zip(gs, results)):
        p0, p1 = int(problem["pose_off"][b]), int(problem["pose_off"][b + 1])
        vp = _T(v_pose[p0:p1])
        vq = None
        if g.is_ba:
            t0, t1 = int(problem["point_off"][b]), int(problem["point_off"][b + 1])
            vq = _T(v_pts[t0:t1]) if v_pts is not None else torch.zeros(t1 - t0, 3, dtype=DT)
        outs.append(implicit_grad_graph(g, r, vp, vq))
    keys = [k for k in outs[0] if k not in ("u", "u_pts")]
    out = {k: torch.cat([o[k] for o in outs]).numpy() for k in keys}
    if all("u" in o for o in outs):
        out["u"] = torch.cat([o["u"].reshape(-1, gs[0].G.dof) for o in outs]).numpy()
    return out


# ---------------------------------------------------------------------------
# large pose graphs: the same steps with a sparse factorisation (Section 4.2)
# ---------------------------------------------------------------------------
def _sparse_factor(H):
    """LU of the symmetric matrix H with a symmetric minimum-degree ordering and
    diagonal pivots (SuperLU), which for a symmetric positive definite matrix
    is its Cholesky factorisation up to the scaling of the factors; a
    non-positive pivot means H is not positive definite.  Returns the factor
    or None."""
    import scipy.sparse.linalg as sla
    try:
        lu = sla.splu(H.tocsc(), permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                      options=dict(SymmetricMode=True))
    except RuntimeError:                      # exactly singular
        return None
    if not np.all(lu.U.diagonal() > 0.0):
        return None
    return lu


def solve_graph_sparse(g: Graph, iterations: int, lam: float, tau=None) -> GraphResult:
    """K fixed-damping steps and the final linearisation of one pose graph,
    as solve_graph (same steps, same order) but with a sparse H and a sparse
    factorisation, for graphs whose dense H does not fit (the 16^3 lattice:
    24576 unknowns).  The result's factor is the sparse factor of H*."""
    if tau is None:
        tau = g.tau
    import scipy.sparse as sp
    X = g.X.clone()
    obj, status = [], OK
    for _ in range(iterations):
        s, H, gv = linearize_pose_graph_sparse(g, X, tau)
        obj.append(s)
        if not (np.isfinite(s) and np.all(np.isfinite(H.data)) and np.all(np.isfinite(gv))):
            status = NONFINITE
            break
        lu = _sparse_factor(H + lam * sp.identity(H.shape[0], format="csr"))
        if lu is None:
            status = NOT_PD
            break
        delta = torch.as_tensor(lu.solve(gv), dtype=DT)
        X = g.G.retract(X, -delta.reshape(-1, g.G.dof))
    res = GraphResult(X=X, pts=None, objective=obj, status=status)
    if status != OK:
        res.objective = obj + [obj[-1]] * (iterations + 1 - len(obj))
        return res
    s, H, gv = linearize_pose_graph_sparse(g, X, tau)
    res.objective = obj + [s]
    res.lin = Lin(S=torch.tensor(s, dtype=DT), H=H, g=torch.as_tensor(gv, dtype=DT))
    if not (np.isfinite(s) and np.all(np.isfinite(H.data)) and np.all(np.isfinite(gv))):
        res.status = NONFINITE
        return res
    lu = _sparse_factor(H)
    res.factor = None if lu is None else (lu,)
    if lu is None:
        res.status = NOT_PD
    return res


def implicit_grad_graph_sparse(g: Graph, res: GraphResult, v_pose) -> dict:
    """Proposition 1 for a result of solve_graph_sparse: u = H*^-1 v with the
    sparse factor, then dL/dphi = -d/dphi [u^T g(theta_K; phi)] by autograd
    of the gradient vector alone (no H)."""
    d = g.G.dof
    if res.status != OK:
        return dict(edge_logw=torch.zeros(len(g.ei), dtype=DT), prior_logw=torch.zeros(len(g.pv), dtype=DT),
                    tau=torch.zeros(len(g.ei), d, dtype=DT))
    (lu,) = res.factor
    u = torch.as_tensor(lu.solve(np.asarray(v_pose, dtype=np.float64).reshape(-1)), dtype=DT)
    le = g.logw_e.clone().requires_grad_(True)
    lp = g.logw_p.clone().requires_grad_(True)
    tau0 = g.tau if g.tau is not None else torch.zeros(len(g.ei), d, dtype=DT)
    tau = tau0.clone().requires_grad_(True)
    _, gvec, _ = objective_and_gradient_pose_graph(g, res.X, tau=tau, logw_e=le, logw_p=lp)
    de, dp, dt = torch.autograd.grad((gvec * u).sum(), [le, lp, tau])
    return dict(edge_logw=-de, prior_logw=-dp, tau=-dt, u=u.reshape(-1, d))


# ---------------------------------------------------------------------------
# outer loss used by the workloads: L = sum_k ||Log(X_gt,k^-1 X_k)||^2
# ---------------------------------------------------------------------------
def pose_error_loss_and_seed(group: str, poses: np.ndarray, poses_gt: np.ndarray):
    """Loss value and its tangent gradient v_k = d/dxi L(X_k Exp(xi)) at xi = 0
    (the right-perturbation gradient of Appendix D, Eq. grad1)."""
    G = lie.group(group)
    X = G.from_storage(_T(poses))
    Xg = G.from_storage(_T(poses_gt))
    xi = torch.zeros(X.shape[0], G.dof, dtype=DT, requires_grad=True)
    e = G.log(G.inv(Xg) @ G.retract(X, xi))
    L = (e ** 2).sum()
    (v,) = torch.autograd.grad(L, [xi])
    return float(L.detach()), v.numpy()
