"""Seeded synthetic workloads for the batched DNLS inner step.

This module only draws random numbers and lays them out; it holds none of
the solver's arithmetic.  Rotations are built with SciPy's ``Rotation``
(a library routine), poses are composed with plain 4x4 / 3x3 homogeneous
matrix products, and every graph ``b`` of workload ``cfg`` draws from
``numpy.random.default_rng(SeedSequence([cfg, b, seed]))`` so any graph can
be regenerated on its own.

The paper evaluates pose-graph optimisation on a synthetic "Cube" dataset
that it describes only qualitatively (odometry with loop closures,
Appendix E.1) and bundle adjustment on public BAL files (Appendix E.3).
Neither generator nor file is available, so the workloads below are
stand-ins with the shapes the paper's experiments use.

Layout (all arrays are numpy, indices are global across the batch):
  group        "SE2" or "SE3"
  pose_off     int32 [B+1]   poses of graph b are pose_off[b]:pose_off[b+1]
  poses_gt     float64 [V,3,4] (SE3: [R|t]) or [V,4] (SE2: x, y, cos, sin)
  poses_init   same shape as poses_gt
  edge_off     int32 [B+1]
  edge_ij      int32 [E,2]   relative-pose measurement from pose i to pose j
  edge_meas    same per-element shape as poses (measured X_i^-1 X_j)
  prior_off    int32 [B+1]
  prior_var    int32 [P]
  prior_meas   same per-element shape as poses
  edge_logw    float64 [E]   log of the scalar cost weight (0 = unit weight)
  prior_logw   float64 [P]
Bundle adjustment adds:
  point_off    int32 [B+1]
  points_gt / points_init   float64 [Vp,3]
  obs_off      int32 [B+1]
  obs_cam, obs_pt  int32 [O]
  obs_uv       float64 [O,2]   measured pixel
  obs_w        float64 [O]     per-observation scalar weight
  intrinsics   (fx, fy, cx, cy); huber_delta float
"""
from __future__ import annotations

import numpy as np
from scipy.spatial.transform import Rotation

__all__ = [
    "circle_se2",
    "walk_se3",
    "uneven_walk_se3",
    "lattice_se3",
    "bundle_adjustment",
    "WORKLOADS",
    "rng_for",
]


def rng_for(cfg: int, b: int, seed: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([cfg, b, seed]))


# --------------------------------------------------------------------------
# homogeneous-matrix helpers (composition only)
# --------------------------------------------------------------------------
def _rot(rotvec: np.ndarray) -> np.ndarray:
    return Rotation.from_rotvec(np.asarray(rotvec, dtype=np.float64)).as_matrix()


def _T3(R: np.ndarray, t: np.ndarray) -> np.ndarray:
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = t
    return T


def _inv3(T: np.ndarray) -> np.ndarray:
    R = T[:3, :3]
    return _T3(R.T, -R.T @ T[:3, 3])


def _noise3(rng, sigma_t: float, sigma_r: float) -> np.ndarray:
    """Perturbation: rotation from a Gaussian rotation vector, Gaussian translation."""
    n_t = rng.normal(0.0, sigma_t, 3)
    n_r = rng.normal(0.0, sigma_r, 3)
    return _T3(_rot(n_r), n_t)


def _T2(x: float, y: float, th: float) -> np.ndarray:
    c, s = np.cos(th), np.sin(th)
    return np.array([[c, -s, x], [s, c, y], [0.0, 0.0, 1.0]])


def _inv2(T: np.ndarray) -> np.ndarray:
    R = T[:2, :2]
    out = np.eye(3)
    out[:2, :2] = R.T
    out[:2, 2] = -R.T @ T[:2, 2]
    return out


def _pack2(T: np.ndarray) -> np.ndarray:
    c, s = T[0, 0], T[1, 0]
    n = np.hypot(c, s)
    return np.array([T[0, 2], T[1, 2], c / n, s / n])


def _pack3(T: np.ndarray) -> np.ndarray:
    return T[:3, :].copy()


def _loop_pairs(rng, n_poses: int, n_loops: int) -> list[tuple[int, int]]:
    """Distinct (i, j) with j - i >= 2, drawn uniformly without replacement."""
    pairs = set()
    max_pairs = (n_poses - 1) * (n_poses - 2) // 2
    n_loops = min(n_loops, max_pairs)
    while len(pairs) < n_loops:
        i, j = sorted(rng.choice(n_poses, size=2, replace=False))
        if j - i >= 2:
            pairs.add((int(i), int(j)))
    return sorted(pairs)


def _concat(graphs: list[dict], group: str) -> dict:
    """Stack per-graph dicts (local indices) into one batch with global indices."""
    out: dict = {"group": group}
    pose_off, edge_off, prior_off = [0], [0], [0]
    keys_pose = ["poses_gt", "poses_init"]
    acc = {k: [] for k in keys_pose + ["edge_ij", "edge_meas", "prior_var", "prior_meas",
                                       "edge_logw", "prior_logw"]}
    for g in graphs:
        base = pose_off[-1]
        for k in keys_pose:
            acc[k].append(g[k])
        acc["edge_ij"].append(g["edge_ij"] + base)
        acc["edge_meas"].append(g["edge_meas"])
        acc["prior_var"].append(g["prior_var"] + base)
        acc["prior_meas"].append(g["prior_meas"])
        acc["edge_logw"].append(np.zeros(len(g["edge_ij"])))
        acc["prior_logw"].append(np.asarray(g.get("prior_logw", np.zeros(len(g["prior_var"])))))
        pose_off.append(base + len(g["poses_gt"]))
        edge_off.append(edge_off[-1] + len(g["edge_ij"]))
        prior_off.append(prior_off[-1] + len(g["prior_var"]))
    for k, v in acc.items():
        out[k] = np.concatenate(v, axis=0)
    out["edge_ij"] = out["edge_ij"].astype(np.int32).reshape(-1, 2)
    out["prior_var"] = out["prior_var"].astype(np.int32)
    out["pose_off"] = np.asarray(pose_off, dtype=np.int32)
    out["edge_off"] = np.asarray(edge_off, dtype=np.int32)
    out["prior_off"] = np.asarray(prior_off, dtype=np.int32)
    return out


# --------------------------------------------------------------------------
# SE(2) circle (one graph, 16 poses)
# --------------------------------------------------------------------------
def circle_se2(batch: int = 1, n_poses: int = 16, n_loops: int = 8, radius: float = 5.0,
               sigma_t: float = 0.05, sigma_th: float = 0.02, noiseless: bool = False,
               cfg: int = 1, seed: int = 0) -> dict:
    """Poses on a circle, heading tangent to it; odometry (k, k+1) plus loop closures."""
    graphs = []
    for b in range(batch):
        rng = rng_for(cfg, b, seed)
        alpha = 2.0 * np.pi * np.arange(n_poses) / n_poses
        gt = [_T2(radius * np.cos(a), radius * np.sin(a), a + np.pi / 2) for a in alpha]
        pairs = [(k, k + 1) for k in range(n_poses - 1)] + _loop_pairs(rng, n_poses, n_loops)
        meas = []
        for (i, j) in pairs:
            Z = _inv2(gt[i]) @ gt[j]
            if not noiseless:
                Z = Z @ _T2(rng.normal(0, sigma_t), rng.normal(0, sigma_t), rng.normal(0, sigma_th))
            meas.append(Z)
        init = [gt[0]]
        for k in range(n_poses - 1):
            init.append(init[-1] @ meas[k])
        graphs.append({
            "poses_gt": np.stack([_pack2(T) for T in gt]),
            "poses_init": np.stack([_pack2(T) for T in init]),
            "edge_ij": np.asarray(pairs, dtype=np.int64),
            "edge_meas": np.stack([_pack2(T) for T in meas]),
            "prior_var": np.asarray([0]),
            "prior_meas": _pack2(gt[0])[None],
        })
    return _concat(graphs, "SE2")


# --------------------------------------------------------------------------
# SE(3) random walks (fixed or uneven sizes)
# --------------------------------------------------------------------------
def _walk_graph(rng, n_poses: int, n_loops: int, sigma_t: float, sigma_r: float,
                noiseless: bool, init_noise: tuple[float, float] | None = None, outliers: int = 0) -> dict:
    gt = [np.eye(4)]
    for _ in range(n_poses - 1):
        step_t = np.array([1.0, 0.0, 0.0]) + 0.2 * rng.normal(size=3)
        step_r = 0.2 * rng.normal(size=3)
        gt.append(gt[-1] @ _T3(_rot(step_r), step_t))
    pairs = [(k, k + 1) for k in range(n_poses - 1)] + _loop_pairs(rng, n_poses, n_loops)
    meas = []
    for (i, j) in pairs:
        Z = _inv3(gt[i]) @ gt[j]
        if not noiseless:
            Z = Z @ _noise3(rng, sigma_t, sigma_r)
        meas.append(Z)
    if init_noise is None:
        init = [gt[0]]
        for k in range(n_poses - 1):
            init.append(init[-1] @ meas[k])
    else:
        init = [gt[0]] + [T @ _noise3(rng, init_noise[0], init_noise[1]) for T in gt[1:]]
    # gross outliers: the first `outliers` loop closures get a random relative
    # pose (drawn last, so the other draws do not depend on the count)
    for q in range(min(outliers, len(pairs) - (n_poses - 1))):
        meas[n_poses - 1 + q] = _T3(_rot(rng.uniform(-np.pi, np.pi, size=3) / np.sqrt(3.0)), rng.normal(0.0, 3.0, size=3))
    return {
        "poses_gt": np.stack([_pack3(T) for T in gt]),
        "poses_init": np.stack([_pack3(T) for T in init]),
        "edge_ij": np.asarray(pairs, dtype=np.int64),
        "edge_meas": np.stack([_pack3(T) for T in meas]),
        "prior_var": np.asarray([0]),
        "prior_meas": _pack3(gt[0])[None],
    }


def walk_se3(batch: int = 128, n_poses: int = 64, n_loops: int = 64, sigma_t: float = 0.05,
             sigma_r: float = 0.01, noiseless: bool = False, init_noise=None,
             cfg: int = 2, seed: int = 0, outliers: int = 0) -> dict:
    """Random-walk trajectories: each step moves about one unit along the body x axis
    with Gaussian jitter (0.2) in translation and rotation vector; odometry edges
    (k, k+1) plus uniformly drawn loop closures; initial guess composed from the
    noisy odometry.  `outliers` loop closures per graph are replaced by random
    relative poses (the loop-closure outliers of a robust-cost experiment)."""
    graphs = [_walk_graph(rng_for(cfg, b, seed), n_poses, n_loops, sigma_t, sigma_r, noiseless,
                          init_noise, outliers) for b in range(batch)]
    return _concat(graphs, "SE3")


def uneven_walk_se3(batch: int = 256, n_min: int = 32, n_max: int = 256, sigma_t: float = 0.05,
                    sigma_r: float = 0.01, noiseless: bool = False, cfg: int = 4,
                    seed: int = 0) -> dict:
    """Random walks whose pose count is uniform in [n_min, n_max], N//2 loop closures."""
    graphs = []
    for b in range(batch):
        rng = rng_for(cfg, b, seed)
        n = int(rng.integers(n_min, n_max + 1))
        graphs.append(_walk_graph(rng, n, n // 2, sigma_t, sigma_r, noiseless))
    return _concat(graphs, "SE3")


# --------------------------------------------------------------------------
# SE(3) lattice (block-sparse workload)
# --------------------------------------------------------------------------
def lattice_se3(batch: int = 8, side: int = 16, long_frac: float = 0.1, sigma_t: float = 0.05,
                sigma_r: float = 0.01, init_t: float = 0.1, init_r: float = 0.05,
                noiseless: bool = False, cfg: int = 3, seed: int = 0) -> dict:
    """Poses at integer points of a side^3 lattice, random orientations, edges to the
    6-neighbourhood plus long_frac x (#lattice edges) uniform non-adjacent pairs;
    initial guess = ground truth perturbed per pose."""
    graphs = []
    n = side ** 3
    for b in range(batch):
        rng = rng_for(cfg, b, seed)
        gt = []
        for c in range(side):
            for bb in range(side):
                for a in range(side):
                    gt.append(_T3(_rot(0.3 * rng.normal(size=3)), np.array([a, bb, c], float)))
        pairs = []
        for k in range(n):
            a, bb, c = k % side, (k // side) % side, k // (side * side)
            if a + 1 < side:
                pairs.append((k, k + 1))
            if bb + 1 < side:
                pairs.append((k, k + side))
            if c + 1 < side:
                pairs.append((k, k + side * side))
        existing = set(pairs)
        n_long = int(round(long_frac * len(pairs)))
        longs = set()
        while len(longs) < n_long:
            i, j = sorted(int(x) for x in rng.choice(n, size=2, replace=False))
            if (i, j) not in existing:
                longs.add((i, j))
        pairs = pairs + sorted(longs)
        meas = []
        for (i, j) in pairs:
            Z = _inv3(gt[i]) @ gt[j]
            if not noiseless:
                Z = Z @ _noise3(rng, sigma_t, sigma_r)
            meas.append(Z)
        init = [gt[0]] + [T @ _noise3(rng, init_t, init_r) for T in gt[1:]]
        graphs.append({
            "poses_gt": np.stack([_pack3(T) for T in gt]),
            "poses_init": np.stack([_pack3(T) for T in init]),
            "edge_ij": np.asarray(pairs, dtype=np.int64),
            "edge_meas": np.stack([_pack3(T) for T in meas]),
            "prior_var": np.asarray([0]),
            "prior_meas": _pack3(gt[0])[None],
        })
    return _concat(graphs, "SE3")


# --------------------------------------------------------------------------
# bundle adjustment
# --------------------------------------------------------------------------
def _look_at(center: np.ndarray, target: np.ndarray) -> np.ndarray:
    """World-to-camera transform of a camera at `center` looking at `target`
    (camera z forward, x right, y down)."""
    z = target - center
    z = z / np.linalg.norm(z)
    up = np.array([0.0, 0.0, 1.0])
    x = np.cross(z, up)
    x = x / np.linalg.norm(x)
    y = np.cross(z, x)
    R_wc = np.stack([x, y, z], axis=1)  # camera axes in world frame
    return _T3(R_wc.T, -R_wc.T @ center)


def bundle_adjustment(batch: int = 4, n_cams: int = 64, n_points: int = 2048,
                      obs_per_point: int = 8, radius: float = 10.0, f: float = 500.0,
                      width: int = 640, height: int = 480, pixel_sigma: float = 1.0,
                      huber_delta: float = 2.0, cam_r: float = 0.02, cam_t: float = 0.05,
                      point_sigma: float = 0.05, prior_w: float = 1e3,
                      noiseless: bool = False, cfg: int = 5, seed: int = 0) -> dict:
    """Cameras on a ring in the z=0 plane facing the origin, Gaussian points,
    each point seen by `obs_per_point` distinct cameras that see it in front
    and inside the image; the first two cameras carry a strong prior."""
    fx = fy = f
    cx, cy = width / 2.0, height / 2.0
    cams_gt, cams_init, pts_gt, pts_init = [], [], [], []
    obs_cam, obs_pt, obs_uv = [], [], []
    prior_var, prior_meas = [], []
    cam_off, pt_off, obs_off, prior_off = [0], [0], [0], [0]
    for b in range(batch):
        rng = rng_for(cfg, b, seed)
        ang = 2.0 * np.pi * np.arange(n_cams) / n_cams
        T = [_look_at(np.array([radius * np.cos(a), radius * np.sin(a), 0.0]), np.zeros(3))
             for a in ang]
        P = rng.normal(size=(n_points, 3))
        cb, pb = cam_off[-1], pt_off[-1]
        for p in range(n_points):
            vis = []
            for c in range(n_cams):
                pc = T[c][:3, :3] @ P[p] + T[c][:3, 3]
                if pc[2] <= 0.1:
                    continue
                u, v = fx * pc[0] / pc[2] + cx, fy * pc[1] / pc[2] + cy
                if 0.0 <= u < width and 0.0 <= v < height:
                    vis.append((c, u, v))
            if len(vis) < obs_per_point:
                raise RuntimeError("point seen by too few cameras")
            pick = rng.choice(len(vis), size=obs_per_point, replace=False)
            for k in sorted(pick):
                c, u, v = vis[k]
                if not noiseless:
                    u, v = u + rng.normal(0, pixel_sigma), v + rng.normal(0, pixel_sigma)
                obs_cam.append(cb + c)
                obs_pt.append(pb + p)
                obs_uv.append((u, v))
        for c in range(n_cams):
            cams_gt.append(_pack3(T[c]))
            if c < 2 or noiseless:
                cams_init.append(_pack3(T[c]))
            else:
                cams_init.append(_pack3(T[c] @ _noise3(rng, cam_t, cam_r)))
        for c in range(2):
            prior_var.append(cb + c)
            prior_meas.append(_pack3(T[c]))
        pts_gt.append(P)
        pts_init.append(P if noiseless else P + rng.normal(0, point_sigma, P.shape))
        cam_off.append(cb + n_cams)
        pt_off.append(pb + n_points)
        obs_off.append(len(obs_cam))
        prior_off.append(len(prior_var))
    return {
        "group": "SE3",
        "pose_off": np.asarray(cam_off, np.int32),
        "poses_gt": np.stack(cams_gt),
        "poses_init": np.stack(cams_init),
        "point_off": np.asarray(pt_off, np.int32),
        "points_gt": np.concatenate(pts_gt),
        "points_init": np.concatenate(pts_init),
        "obs_off": np.asarray(obs_off, np.int32),
        "obs_cam": np.asarray(obs_cam, np.int32),
        "obs_pt": np.asarray(obs_pt, np.int32),
        "obs_uv": np.asarray(obs_uv, np.float64),
        "obs_w": np.ones(len(obs_cam)),
        "intrinsics": (fx, fy, cx, cy),
        "huber_delta": float(huber_delta),
        "edge_off": np.zeros(batch + 1, np.int32),
        "edge_ij": np.zeros((0, 2), np.int32),
        "edge_meas": np.zeros((0, 3, 4)),
        "edge_logw": np.zeros(0),
        "prior_off": np.asarray(prior_off, np.int32),
        "prior_var": np.asarray(prior_var, np.int32),
        "prior_meas": np.stack(prior_meas),
        "prior_logw": np.full(len(prior_var), np.log(prior_w)),
    }


# Named workloads with the sizes of the five evaluation configurations.
WORKLOADS = {
    "se2_circle_b1": dict(fn=circle_se2, kwargs=dict(batch=1), iterations=10, optimizer="GN",
                          lam=0.0, solver="dense", precision="fp64"),
    "se3_walk64_b128": dict(fn=walk_se3, kwargs=dict(batch=128), iterations=10, optimizer="LM",
                            lam=1e-3, solver="dense", precision="mixed"),
    "se3_lattice16_b8": dict(fn=lattice_se3, kwargs=dict(batch=8), iterations=15, optimizer="GN",
                             lam=0.0, solver="sparse", precision="mixed"),
    "se3_uneven_b256": dict(fn=uneven_walk_se3, kwargs=dict(batch=256), iterations=10,
                            optimizer="GN", lam=0.0, solver="sparse", precision="mixed"),
    "ba_ring64_b4": dict(fn=bundle_adjustment, kwargs=dict(batch=4), iterations=10,
                         optimizer="LM", lam=1e-3, solver="schur", precision="mixed"),
}
