"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and the bench.

This module only draws random inputs and lays them out in memory.  It holds none of
the renderer's arithmetic (no decode, projection, binning, compositing, loss or
gradient): both the FP64 oracle and the HIP path consume what it produces.

The paper's workloads are outdoor driving sequences (KITTI, Oxford RobotCar, Malaga;
Sec. IV-A).  None of that data is here.  The street-like "corridor" scenes below stand
in for the shape of those workloads: a road plane with two facades, anchors snapped to
a voxel grid as in the voxelisation of Eq. 4 (Sec. III-B), with the voxel size set to
0.2 m, KITTI-like 1226x370 views with fx = fy = 718.

Layouts (all float32 unless stated):
  plain scene   mean[3][G], log_scale[3][G], quat[4][G] (w,x,y,z, not normalised),
                logit[G], rgb[3][G]
  anchors       pos[3][A], feat[A][F], log_scale[A], offs[3][A*K] (index a*K + j),
                part_begin[M+1] (int32, anchors grouped by partition)
  mlp           [M][P] per partition, three two-layer MLPs packed in the order
                (opacity, colour, covariance), each as W1[hidden][F+4], b1[hidden],
                W2[out][hidden], b2[out] with out = K, 3K, 7K
  camera        dict: R (3x3 world->camera, row-major), t (3), fx, fy, cx, cy, W, H,
                partition; OpenCV axes (x right, y down, z forward)
  target        [3][H][W] per view
"""
from __future__ import annotations

import math

import numpy as np

VOXEL = 0.2  # metres; the corridor generator's voxel size


def mlp_param_count(F: int, K: int, hidden: int = 32) -> int:
    n_in = F + 4
    total = 0
    for out in (K, 3 * K, 7 * K):
        total += hidden * n_in + hidden + out * hidden + out
    return total


def _xavier(rng, fan_out, fan_in):
    b = math.sqrt(6.0 / (fan_in + fan_out))
    return rng.uniform(-b, b, size=(fan_out, fan_in))


def random_mlp(rng, F: int, K: int, hidden: int = 32, bias_std: float = 0.0) -> np.ndarray:
    """Xavier-uniform (gain 1) weights; biases zero unless bias_std > 0 (tests only)."""
    n_in = F + 4
    parts = []
    for out in (K, 3 * K, 7 * K):
        parts.append(_xavier(rng, hidden, n_in).ravel())
        parts.append(rng.normal(0.0, bias_std, hidden) if bias_std > 0 else np.zeros(hidden))
        parts.append(_xavier(rng, out, hidden).ravel())
        parts.append(rng.normal(0.0, bias_std, out) if bias_std > 0 else np.zeros(out))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == mlp_param_count(F, K, hidden)
    return p


def camera(R, t, fx, fy, cx, cy, W, H, partition=0) -> dict:
    return dict(R=np.asarray(R, np.float32).reshape(3, 3), t=np.asarray(t, np.float32).reshape(3),
                fx=float(fx), fy=float(fy), cx=float(cx), cy=float(cy), W=int(W), H=int(H),
                partition=int(partition))


def _yaw(psi):
    c, s = math.cos(psi), math.sin(psi)
    # rotation about the camera y axis (camera-to-world for a yawed camera)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def posed_camera(centre, cam_to_world, fx, fy, cx, cy, W, H, partition=0) -> dict:
    """World->camera pose from a camera centre and a camera-to-world rotation."""
    Rwc = np.asarray(cam_to_world, np.float64).T
    t = -Rwc @ np.asarray(centre, np.float64)
    return camera(Rwc, t, fx, fy, cx, cy, W, H, partition)


# ----------------------------------------------------------------------------------
# Config 1: plain Gaussians, no anchors
# ----------------------------------------------------------------------------------

def plain_scene(seed: int = 1001, G: int = 1000, W: int = 64, H: int = 48,
                fx: float = 60.0, fy: float = 60.0, cx: float | None = None,
                cy: float | None = None) -> dict:
    rng = np.random.default_rng(seed)
    cx = W / 2 if cx is None else cx
    cy = H / 2 if cy is None else cy
    mean = np.stack([rng.uniform(-3, 3, G), rng.uniform(-2, 2, G), rng.uniform(2, 10, G)])
    log_scale = rng.normal(-2.5, 0.5, (3, G))
    quat = rng.normal(0.0, 1.0, (4, G))
    logit = rng.normal(0.0, 1.0, G)
    rgb = rng.uniform(0.0, 1.0, (3, G))
    cam = camera(np.eye(3), np.zeros(3), fx, fy, cx, cy, W, H)
    target = rng.uniform(0.0, 1.0, (3, H, W))
    f32 = lambda a: np.ascontiguousarray(a, np.float32)
    return dict(kind="plain", mean=f32(mean), log_scale=f32(log_scale), quat=f32(quat),
                logit=f32(logit), rgb=f32(rgb), cams=[cam], targets=[f32(target)],
                ssim_weight=0.0, opacity_mode="sigmoid")


# ----------------------------------------------------------------------------------
# Corridor voxels: road plane 1.6 m below the camera, facades at x = +-8 m
# ----------------------------------------------------------------------------------

def corridor_voxels(z0: float = 2.0, z1: float = 80.0, half_width: float = 8.0,
                    ground_y: float = 1.6, wall_height: float = 6.0, eps: float = VOXEL) -> np.ndarray:
    """Unique voxel centres (integer lattice coordinates times eps) on the corridor
    surfaces, in the frame of a camera at the origin looking along +z.  Returns [N][3]."""
    ix = np.arange(round(-half_width / eps), round(half_width / eps) + 1)
    iz = np.arange(round(z0 / eps), round(z1 / eps) + 1)
    iy_ground = round(ground_y / eps)
    iy = np.arange(round((ground_y - wall_height) / eps), iy_ground + 1)
    g = np.stack(np.meshgrid(ix, [iy_ground], iz, indexing="ij"), -1).reshape(-1, 3)
    walls = []
    for sx in (ix[0], ix[-1]):
        walls.append(np.stack(np.meshgrid([sx], iy, iz, indexing="ij"), -1).reshape(-1, 3))
    lattice = np.unique(np.concatenate([g] + walls), axis=0)
    return lattice.astype(np.float64) * eps


def corridor_anchors(rng, A: int, F: int = 32, K: int = 10, voxels: np.ndarray | None = None):
    vox = corridor_voxels() if voxels is None else voxels
    if A > len(vox):
        raise ValueError(f"{A} anchors requested, corridor holds {len(vox)} voxels")
    idx = np.sort(rng.choice(len(vox), size=A, replace=False))
    pos = vox[idx].T
    feat = rng.normal(0.0, 1.0, (A, F))
    log_scale = rng.normal(-2.0, 0.3, A)
    offs = rng.normal(0.0, 0.1, (3, A * K))
    return pos, feat, log_scale, offs


def corridor_views(rng, n_views: int, W: int, H: int, fx: float = 718.0, fy: float = 718.0,
                   spacing: float = 1.0, yaw_deg: float = 2.0, partition: int = 0,
                   jitter: bool = True) -> list:
    cams = []
    for i in range(n_views):
        psi = math.radians(rng.uniform(-yaw_deg, yaw_deg)) if jitter else 0.0
        cams.append(posed_camera([0.0, 0.0, i * spacing], _yaw(psi), fx, fy, W / 2, H / 2, W, H,
                                 partition))
    return cams


def anchor_scene(seed: int, anchors_per_part, views_per_part: int, W: int = 1226, H: int = 370,
                 fx: float = 718.0, F: int = 32, K: int = 10, hidden: int = 32,
                 ssim_weight: float = 0.0, jitter: bool = True, bias_std: float = 0.0,
                 per_part_seed: bool = True) -> dict:
    """Anchor scene with one independent corridor and MLP set per partition."""
    anchors_per_part = list(anchors_per_part)
    M = len(anchors_per_part)
    pos, feat, ls, offs, mlps, cams, targets = [], [], [], [], [], [], []
    vox = corridor_voxels()
    base = np.random.default_rng(seed)
    for m, A in enumerate(anchors_per_part):
        rng = np.random.default_rng(seed + 100 * m) if per_part_seed else base
        p, f, l, o = corridor_anchors(rng, A, F, K, vox)
        pos.append(p); feat.append(f); ls.append(l); offs.append(o.reshape(3, A, K))
        mlps.append(random_mlp(rng, F, K, hidden, bias_std))
        if views_per_part == 1 and not jitter:
            vc = [camera(np.eye(3), np.zeros(3), fx, fx, W / 2, H / 2, W, H, m)]
        else:
            vc = corridor_views(rng, views_per_part, W, H, fx, fx, partition=m, jitter=jitter)
        cams.extend(vc)
        for _ in vc:
            targets.append(rng.uniform(0.0, 1.0, (3, H, W)).astype(np.float32))
    f32 = lambda a: np.ascontiguousarray(a, np.float32)
    A_tot = sum(anchors_per_part)
    part_begin = np.concatenate([[0], np.cumsum(anchors_per_part)]).astype(np.int32)
    return dict(kind="anchor", F=F, K=K, hidden=hidden,
                pos=f32(np.concatenate(pos, 1)), feat=f32(np.concatenate(feat, 0)),
                log_scale=f32(np.concatenate(ls)),
                offs=f32(np.concatenate(offs, 1).reshape(3, A_tot * K)),
                part_begin=part_begin, mlp=f32(np.stack(mlps)), cams=cams, targets=targets,
                ssim_weight=ssim_weight, opacity_mode="tanh")


def log_uniform_counts(rng, n: int, lo: float, hi: float, div: int = 10) -> list:
    g = np.exp(rng.uniform(math.log(lo), math.log(hi), n))
    return [int(round(x / div)) for x in g]


# ----------------------------------------------------------------------------------
# Named configurations
# ----------------------------------------------------------------------------------

def config(name: str) -> dict:
    """The five workloads: C1 plain 1k Gaussians at 64x48; C2 20k anchors, 1 view at
    1226x370; C3 50k anchors, 4 views, L1 + 0.2 (1 - SSIM); C4 16 partitions x 4 views
    with log-uniform anchor counts; C5 the 2 km path (see long_path_scene)."""
    if name == "C1":
        return plain_scene(1001)
    if name == "C2":
        return anchor_scene(1002, [20000], 1, jitter=False)
    if name == "C3":
        return anchor_scene(1003, [50000], 4, ssim_weight=0.2)
    if name == "C4":
        counts = log_uniform_counts(np.random.default_rng(1004), 16, 20e3, 400e3)
        return anchor_scene(1004, counts, 4, ssim_weight=0.2)
    if name == "C5":
        return long_path_scene(1005)
    raise KeyError(name)


def one_view(scene: dict, v: int) -> dict:
    """The single-view workload of view v of an anchor scene (one mapping iteration on one
    keyframe): the whole scene's anchors and MLP sets, that view's camera and target."""
    sub = dict(scene)
    sub.update(cams=[scene["cams"][v]], targets=[scene["targets"][v]])
    return sub


def long_path_scene(seed: int = 1005, n_parts: int = 64, views_per_part: int = 8,
                    F: int = 32, K: int = 10, hidden: int = 32, with_targets: bool = True) -> dict:
    """2 km polyline of five 400 m straight segments with alternating 90-degree turns.
    Partition p has its keyframe at arc length p * 31.25 m and draws its anchors from the
    voxels of its look-ahead window [s+2, s+80] m (the corridor cross-section in the
    local segment frame); its 8 views sit at s + j * 3.906 m with +-2 deg yaw jitter and
    cycle through 1226x370, 1280x384 and 1280x960."""
    rng0 = np.random.default_rng(seed)
    counts = log_uniform_counts(rng0, n_parts, 30e3, 300e3)
    seg_len = 400.0
    heading = [0.0]
    for i in range(1, 5):
        heading.append(heading[-1] + (math.pi / 2 if i % 2 else -math.pi / 2))
    starts = [np.zeros(2)]
    for i in range(4):
        d = np.array([math.sin(heading[i]), math.cos(heading[i])])
        starts.append(starts[-1] + seg_len * d)

    def frame_at(s):
        i = min(int(s // seg_len), 4)
        d = np.array([math.sin(heading[i]), math.cos(heading[i])])
        p = starts[i] + (s - i * seg_len) * d
        return np.array([p[0], 0.0, p[1]]), heading[i]

    local = corridor_voxels(0.0, 78.0)  # window relative to the keyframe, z in [0, 78]
    res = [(1226, 370), (1280, 384), (1280, 960)]
    pos, feat, ls, offs, mlps, cams, targets = [], [], [], [], [], [], []
    vi = 0
    for p in range(n_parts):
        rng = np.random.default_rng(seed + 100 * p)
        s0 = p * 31.25
        origin, h = frame_at(s0 + 2.0)
        rot = _yaw(h)
        A = counts[p]
        idx = np.sort(rng.choice(len(local), size=A, replace=False))
        world = (rot @ local[idx].T) + origin[:, None]
        pos.append(world)
        feat.append(rng.normal(0.0, 1.0, (A, F)))
        ls.append(rng.normal(-2.0, 0.3, A))
        offs.append(rng.normal(0.0, 0.1, (3, A, K)))
        mlps.append(random_mlp(rng, F, K, hidden))
        for j in range(views_per_part):
            c, hj = frame_at(s0 + j * 3.906)
            psi = math.radians(rng.uniform(-2.0, 2.0))
            W, H = res[vi % 3]
            vi += 1
            cams.append(posed_camera(c, _yaw(hj + psi), 718.0, 718.0, W / 2, H / 2, W, H, p))
            if with_targets:
                targets.append(rng.uniform(0.0, 1.0, (3, H, W)).astype(np.float32))
    f32 = lambda a: np.ascontiguousarray(a, np.float32)
    A_tot = sum(counts)
    return dict(kind="anchor", F=F, K=K, hidden=hidden,
                pos=f32(np.concatenate(pos, 1)), feat=f32(np.concatenate(feat, 0)),
                log_scale=f32(np.concatenate(ls)),
                offs=f32(np.concatenate(offs, 1).reshape(3, A_tot * K)),
                part_begin=np.concatenate([[0], np.cumsum(counts)]).astype(np.int32),
                mlp=f32(np.stack(mlps)), cams=cams, targets=targets, ssim_weight=0.2,
                opacity_mode="tanh")

# ----------------------------------------------------------------------------------
# Loop-closure corrections: keyframes along the corridor and small pose corrections
# ----------------------------------------------------------------------------------

def _axis_angle(axis, angle):
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    return np.eye(3) + math.sin(angle) * K + (1.0 - math.cos(angle)) * (K @ K)


def loop_fixes(seed: int, n: int, W: int = 1226, H: int = 370, spacing: float = 3.0, rot_deg: float = 1.0,
               trans_m: float = 0.1) -> list:
    """n keyframes along the corridor (old poses) with random corrections of up to rot_deg
    degrees about a random axis and trans_m metres: dicts with R_old, t_old, R_new, t_new
    (world->camera) and the intrinsics."""
    rng = np.random.default_rng(seed)
    out = []
    for i, c in enumerate(corridor_views(rng, n, W, H, spacing=spacing)):
        dR = _axis_angle(rng.normal(size=3), math.radians(rng.uniform(-rot_deg, rot_deg)))
        R_new = (dR @ c["R"].astype(np.float64)).astype(np.float32)
        t_new = (c["t"] + rng.uniform(-trans_m, trans_m, 3)).astype(np.float32)
        out.append(dict(R_old=c["R"], t_old=c["t"], R_new=R_new, t_new=t_new, fx=c["fx"], fy=c["fy"],
                        cx=c["cx"], cy=c["cy"], W=c["W"], H=c["H"]))
    return out

# ----------------------------------------------------------------------------------
# Flow correspondences between two keyframes of the corridor
# ----------------------------------------------------------------------------------

def flow_pairs(seed: int, n: int, baseline: float = 1.0, noise_px: float = 0.0, outlier_frac: float = 0.0,
               W: int = 1226, H: int = 370):
    """Correspondences x1 <-> x2 of n corridor surface points seen by two keyframes
    `baseline` metres apart along the corridor (yaw jitter as the keyframes of the
    workloads), with Gaussian pixel noise on x2 and a fraction of outliers (x2 replaced by
    a uniform random pixel).  Returns (cam1, cam2, x1 [2][n], x2 [2][n] float32, points
    [3][n] float64, outlier mask)."""
    rng = np.random.default_rng(seed)
    cams = corridor_views(rng, 2, W, H, spacing=baseline)
    vox = corridor_voxels(z0=baseline + 3.0, z1=80.0)
    pts = vox[rng.choice(len(vox), n, replace=True)] + rng.uniform(-0.1, 0.1, (n, 3))
    out = []
    for c in cams:
        y = c["R"].astype(np.float64) @ pts.T + c["t"].astype(np.float64)[:, None]
        out.append(np.stack([c["fx"] * y[0] / y[2] + c["cx"], c["fy"] * y[1] / y[2] + c["cy"]]))
    x1, x2 = out
    x2 = x2 + rng.normal(0.0, noise_px, x2.shape) if noise_px > 0 else x2
    bad = rng.uniform(size=n) < outlier_frac
    x2[:, bad] = np.stack([rng.uniform(0, W, bad.sum()), rng.uniform(0, H, bad.sum())])
    return cams[0], cams[1], x1.astype(np.float32), x2.astype(np.float32), pts.T, bad



def fused_points(seed: int, n: int, dup_frac: float = 0.3, dup_jitter: float = 2e-4, nan_frac: float = 0.0,
                 far_frac: float = 0.0, far: float = 2.0e3, origin=(0.0, 0.0, 0.0)) -> np.ndarray:
    """A keyframe's fused point cloud [3][n] float32 (tracked plus triangulated flow
    points): points on the corridor surfaces (positions of the corridor lattice plus a
    uniform jitter of +-0.1 m, so the surfaces are covered continuously), shifted by
    origin.  A fraction dup_frac repeats an earlier point with a uniform jitter of
    +-dup_jitter m per axis (the same surface point seen again), nan_frac columns are NaN
    (rejected triangulations) and far_frac points lie +-far m away on every axis (beyond
    a 1 mm grid's key range)."""
    rng = np.random.default_rng(seed)
    vox = corridor_voxels()
    pts = vox[rng.integers(0, len(vox), n)] + rng.uniform(-0.1, 0.1, (n, 3)) + np.asarray(origin, np.float64)
    if n > 1:
        dup = np.flatnonzero(rng.uniform(size=n) < dup_frac)
        dup = dup[dup > 0]
        src = (rng.uniform(size=len(dup)) * dup).astype(np.int64)  # an earlier point
        pts[dup] = pts[src] + rng.uniform(-dup_jitter, dup_jitter, (len(dup), 3))
    far_m = rng.uniform(size=n) < far_frac
    pts[far_m] = rng.choice([-far, far], (int(far_m.sum()), 3))
    pts[rng.uniform(size=n) < nan_frac] = np.nan
    return np.ascontiguousarray(pts.T.astype(np.float32))
