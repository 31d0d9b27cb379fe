"""Seeded synthetic bundle-adjustment windows.

This module simulates a scene and a camera; it holds none of the solver's
arithmetic (no residual Jacobians, no normal equations, no solve).  Both the
FP64 CPU oracle and the HIP path consume exactly the arrays produced here.

Scene model (stands in for the paper's datasets, which are not available):
  * pinhole camera fx = fy = 320, cx = 320, cy = 240, image 640 x 480;
  * camera a has centre c_a = (0, 0, 0.1 a) m (forward motion along +z) and a
    camera-to-world rotation Exp(phi_a) with phi_a ~ N(0, (1 deg)^2 I),
    i.i.d. per frame; the stored pose is world-to-camera (R_a^T, -R_a^T c_a),
    matching the paper's reprojection T_j T_i^{-1} (Sec. 3, Eq. 2);
  * each frame sources `ppf` patches with centres uniform over the image and
    true inverse depth U[0.2, 1.0] (random patch sampling, Sec. 3
    "Patch Extraction"; 96 / 48 patches per frame, Sec. 4 Default / Fast);
  * the patch graph joins each patch to every frame within `radius` of its
    source frame, self-edge included (Sec. 3 "Patch Graph");
  * targets are the true projection of the patch centre plus N(0, 1) px noise
    and weights are U[0.1, 1] per coordinate (the factor head's sigmoid-bounded
    confidence, Sec. 3.1); a chosen fraction of edges are outliers with
    N(0, 20^2) px offsets and weights U[0, 0.05];
  * initial state: the first `n_fixed` poses at truth, others with centre
    noise N(0, 0.05^2) m and rotation noise Exp(N(0, (1 deg)^2)); initial
    inverse depth = truth * U[0.8, 1.2];
  * hidden edges: when the point is behind or too close to camera j, either at
    the truth or at the initial state (depth ratio below 0.5), the edge keeps
    its slot in the graph but gets weight 0 and the anchor pixel as target.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

FX = FY = 320.0
CX, CY = 320.0, 240.0
WIDTH, HEIGHT = 640, 480
HIDE_RATIO = 0.5


@dataclasses.dataclass
class Window:
    """One BA window.  All frame / patch indices are window-local."""
    poses: np.ndarray          # [N,7] f64 initial state, (tx,ty,tz,qx,qy,qz,qw) world->camera
    patches: np.ndarray        # [M,3] f64 (x, y, inverse depth) in the source frame
    anchor: np.ndarray         # [M] int32 source frame of each patch
    kk: np.ndarray             # [E] int32 patch of each edge
    jj: np.ndarray             # [E] int32 target frame of each edge
    targets: np.ndarray        # [E,2] f64 target pixel (values f32-exact when fp32=True)
    weights: np.ndarray        # [E,2] f64 per-coordinate confidence (f32-exact when fp32=True)
    intrinsics: np.ndarray     # [4] f64 fx, fy, cx, cy
    n_fixed: int
    poses_gt: np.ndarray       # [N,7] f64 ground truth
    depth_gt: np.ndarray       # [M] f64 ground-truth inverse depth
    fp32: bool = False

    @property
    def n_frames(self) -> int:
        return int(self.poses.shape[0])

    @property
    def n_patches(self) -> int:
        return int(self.patches.shape[0])

    @property
    def n_edges(self) -> int:
        return int(self.kk.shape[0])

    def copy(self) -> "Window":
        return dataclasses.replace(self, **{f.name: (getattr(self, f.name).copy()
                                   if isinstance(getattr(self, f.name), np.ndarray)
                                   else getattr(self, f.name))
                                   for f in dataclasses.fields(self)})


# ---------------------------------------------------------------- scene helpers
def _rotvec_to_matrix(phi: np.ndarray) -> np.ndarray:
    """Rotation matrix of a rotation vector (scene synthesis only)."""
    th = float(np.linalg.norm(phi))
    if th < 1e-12:
        return np.eye(3)
    k = phi / th
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * (K @ K)


def _matrix_to_quat(R: np.ndarray) -> np.ndarray:
    """(x, y, z, w) unit quaternion with w >= 0 (scene synthesis only)."""
    tr = np.trace(R)
    if tr > 0:
        s = np.sqrt(tr + 1.0) * 2
        w = 0.25 * s
        x = (R[2, 1] - R[1, 2]) / s
        y = (R[0, 2] - R[2, 0]) / s
        z = (R[1, 0] - R[0, 1]) / s
    elif R[0, 0] > R[1, 1] and R[0, 0] > R[2, 2]:
        s = np.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2]) * 2
        w = (R[2, 1] - R[1, 2]) / s
        x = 0.25 * s
        y = (R[0, 1] + R[1, 0]) / s
        z = (R[0, 2] + R[2, 0]) / s
    elif R[1, 1] > R[2, 2]:
        s = np.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2]) * 2
        w = (R[0, 2] - R[2, 0]) / s
        x = (R[0, 1] + R[1, 0]) / s
        y = 0.25 * s
        z = (R[1, 2] + R[2, 1]) / s
    else:
        s = np.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1]) * 2
        w = (R[1, 0] - R[0, 1]) / s
        x = (R[0, 2] + R[2, 0]) / s
        y = (R[1, 2] + R[2, 1]) / s
        z = 0.25 * s
    q = np.array([x, y, z, w])
    q /= np.linalg.norm(q)
    return q if q[3] >= 0 else -q


def _camera(centre: np.ndarray, R_cw: np.ndarray) -> np.ndarray:
    """World->camera pose 7-vector of a camera with centre `centre` and
    camera->world rotation R_cw."""
    R_wc = R_cw.T
    t = -R_wc @ centre
    return np.concatenate([t, _matrix_to_quat(R_wc)])


def _pose_parts(pose: np.ndarray):
    x, y, z, w = pose[3:]
    R = np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
    return R, pose[:3]


def scene_points(poses: np.ndarray, patches: np.ndarray, anchor: np.ndarray,
                 intr: np.ndarray) -> np.ndarray:
    """World points of the patch centres: back-project pixel (x, y) of the
    source camera to metric depth 1/d.  Returns [M,3]."""
    fx, fy, cx, cy = intr
    out = np.empty((patches.shape[0], 3))
    for a in np.unique(anchor):
        sel = anchor == a
        R, t = _pose_parts(poses[a])
        x, y, d = patches[sel, 0], patches[sel, 1], patches[sel, 2]
        ray = np.stack([(x - cx) / fx, (y - cy) / fy, np.ones_like(x)], 1)
        Xc = ray / d[:, None]
        out[sel] = (Xc - t) @ R          # R^T (Xc - t), row-vector form
    return out


def camera_observation(poses: np.ndarray, Xw: np.ndarray, frames: np.ndarray,
                       intr: np.ndarray):
    """Pixel and camera-frame depth of world points Xw[e] seen by camera
    frames[e]."""
    fx, fy, cx, cy = intr
    uv = np.empty((Xw.shape[0], 2))
    depth = np.empty(Xw.shape[0])
    for a in np.unique(frames):
        sel = frames == a
        R, t = _pose_parts(poses[a])
        Xc = Xw[sel] @ R.T + t
        depth[sel] = Xc[:, 2]
        with np.errstate(divide="ignore", invalid="ignore"):
            uv[sel, 0] = fx * Xc[:, 0] / Xc[:, 2] + cx
            uv[sel, 1] = fy * Xc[:, 1] / Xc[:, 2] + cy
    return uv, depth


# ---------------------------------------------------------------- generator
def make_window(n_frames: int, ppf: int, radius: int, *, seed: Sequence[int],
                outlier_frac: float = 0.0, n_fixed: int = 2,
                noise_px: float = 1.0, pose_noise_m: float = 0.05,
                rot_noise_deg: float = 1.0, depth_noise: float = 0.2,
                fp32: bool = False, exact: bool = False) -> Window:
    """Build one synthetic window.

    `exact=True` gives exact-correspondence targets (no pixel noise, no
    outliers, weights still random) so that the truth is a zero-residual
    solution."""
    rng = np.random.default_rng(list(seed))
    intr = np.array([FX, FY, CX, CY])
    deg = np.pi / 180.0

    centres = np.stack([np.array([0.0, 0.0, 0.1 * a]) for a in range(n_frames)])
    R_cw = [_rotvec_to_matrix(rng.normal(0.0, 1.0 * deg, 3)) for _ in range(n_frames)]
    poses_gt = np.stack([_camera(centres[a], R_cw[a]) for a in range(n_frames)])

    M = n_frames * ppf
    anchor = np.repeat(np.arange(n_frames, dtype=np.int32), ppf)
    xy = np.stack([rng.uniform(0, WIDTH, M), rng.uniform(0, HEIGHT, M)], 1)
    depth_gt = rng.uniform(0.2, 1.0, M)

    kk_l, jj_l = [], []
    for k in range(M):
        i = int(anchor[k])
        for j in range(max(0, i - radius), min(n_frames - 1, i + radius) + 1):
            kk_l.append(k)
            jj_l.append(j)
    kk = np.asarray(kk_l, dtype=np.int32)
    jj = np.asarray(jj_l, dtype=np.int32)
    E = kk.shape[0]

    patches_gt = np.concatenate([xy, depth_gt[:, None]], 1)
    Xw = scene_points(poses_gt, patches_gt, anchor, intr)
    uv_true, depth_true = camera_observation(poses_gt, Xw[kk], jj, intr)

    noise = rng.normal(0.0, noise_px, (E, 2))
    weights = rng.uniform(0.1, 1.0, (E, 2))
    n_out = int(round(outlier_frac * E))
    out_idx = rng.choice(E, n_out, replace=False) if n_out > 0 else np.zeros(0, np.int64)
    out_noise = rng.normal(0.0, 20.0, (n_out, 2))
    out_w = rng.uniform(0.0, 0.05, (n_out, 2))
    if exact:
        targets = uv_true.copy()
    else:
        targets = uv_true + noise
        targets[out_idx] = uv_true[out_idx] + out_noise
        weights[out_idx] = out_w

    # initial state
    poses0 = poses_gt.copy()
    for a in range(n_fixed, n_frames):
        c = centres[a] + rng.normal(0.0, pose_noise_m, 3)
        Rn = _rotvec_to_matrix(rng.normal(0.0, rot_noise_deg * deg, 3)) @ R_cw[a]
        poses0[a] = _camera(c, Rn)
    depth0 = depth_gt * rng.uniform(1.0 - depth_noise, 1.0 + depth_noise, M)
    patches0 = np.concatenate([xy, depth0[:, None]], 1)

    # hidden edges: depth ratio (depth in j) / (depth in i) below HIDE_RATIO
    Xw0 = scene_points(poses0, patches0, anchor, intr)
    _, depth_init = camera_observation(poses0, Xw0[kk], jj, intr)
    ratio_true = depth_true * depth_gt[kk]
    ratio_init = depth_init * depth0[kk]
    hidden = (ratio_true < HIDE_RATIO) | (ratio_init < HIDE_RATIO)
    targets[hidden] = xy[kk[hidden]]
    weights[hidden] = 0.0

    if fp32:
        targets = targets.astype(np.float32).astype(np.float64)
        weights = weights.astype(np.float32).astype(np.float64)

    return Window(poses=poses0, patches=patches0, anchor=anchor, kk=kk, jj=jj,
                  targets=targets, weights=weights, intrinsics=intr,
                  n_fixed=min(n_fixed, n_frames), poses_gt=poses_gt,
                  depth_gt=depth_gt, fp32=fp32)


# ---------------------------------------------------------------- named workloads
def plain_fp64_window(window_id: int = 0) -> Window:
    """8 frames x 16 patches, radius 3, no outliers, FP64 path."""
    return make_window(8, 16, 3, seed=[2208, 0, window_id], outlier_frac=0.0)


def method_scale_window(window_id: int = 0) -> Window:
    """22 frames x 96 patches, radius 13, 10% outliers, FP32-rounded inputs."""
    return make_window(22, 96, 13, seed=[2208, 1, window_id], outlier_frac=0.1, fp32=True)


def serving_window(window_id: int) -> Window:
    """Uneven window of a camera stream: frames U{8..22}, patches per frame
    U{48..96}, radius min(13, frames-1), 10% outliers, FP32-rounded inputs."""
    rng = np.random.default_rng([2208, 2, window_id, 7])
    n = int(rng.integers(8, 23))
    ppf = int(rng.integers(48, 97))
    return make_window(n, ppf, min(13, n - 1), seed=[2208, 2, window_id],
                       outlier_frac=0.1, fp32=True)


def gradient_subwindow(window_id: int = 0) -> Window:
    """6 frames x 8 patches, radius 5: the finite-difference gradient case."""
    return make_window(6, 8, 5, seed=[2208, 3, window_id], outlier_frac=0.1, fp32=True)


def large_window(window_id: int = 0) -> Window:
    """64 frames x 256 patches, radius 16, 10% outliers, FP32-rounded inputs."""
    return make_window(64, 256, 16, seed=[2208, 4, window_id], outlier_frac=0.1, fp32=True)


def shuffled(w: Window, seed: int) -> Window:
    """Same window with its edges in a random order (patches untouched)."""
    rng = np.random.default_rng(seed)
    p = rng.permutation(w.n_edges)
    out = w.copy()
    out.kk, out.jj = w.kk[p].copy(), w.jj[p].copy()
    out.targets, out.weights = w.targets[p].copy(), w.weights[p].copy()
    return out


def concat(windows: List[Window]):
    """Offsets for a batch of windows: (frame_off, patch_off, edge_off)."""
    fo = np.zeros(len(windows) + 1, np.int64)
    po = np.zeros(len(windows) + 1, np.int64)
    eo = np.zeros(len(windows) + 1, np.int64)
    for i, w in enumerate(windows):
        fo[i + 1] = fo[i] + w.n_frames
        po[i + 1] = po[i] + w.n_patches
        eo[i + 1] = eo[i] + w.n_edges
    return fo, po, eo


def camera_centres(poses: np.ndarray) -> np.ndarray:
    """Camera centres -R^T t of world->camera poses [N,7]."""
    return np.stack([-_pose_parts(p)[0].T @ p[:3] for p in poses])


def rotation_error_deg(pa: np.ndarray, pb: np.ndarray) -> np.ndarray:
    """Angle of R_a R_b^T in degrees, per frame."""
    out = []
    for a, b in zip(pa, pb):
        M = _pose_parts(a)[0] @ _pose_parts(b)[0].T
        c = (np.trace(M) - 1.0) / 2.0
        v = np.array([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]])
        out.append(np.degrees(np.arctan2(np.linalg.norm(v) / 2.0, c)))
    return np.asarray(out)


def pose_errors(pa: np.ndarray, pb: np.ndarray):
    """(max centre distance in m, max rotation angle in deg) between two pose sets."""
    dc = np.linalg.norm(camera_centres(pa) - camera_centres(pb), axis=1)
    return float(dc.max()) if dc.size else 0.0, float(rotation_error_deg(pa, pb).max()) if len(pa) else 0.0


# ---------------------------------------------------------------- correlation workloads
FEATURE_STRIDE = 4      # the matching features are at 1/4 of the image resolution
FEATURE_DIM = 128       # matching-feature channels


def bf16_exact(a: np.ndarray) -> np.ndarray:
    """float32 values representable in bfloat16 (round to nearest even), so
    the same numbers feed a bf16 buffer and a float64 reference."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def bf16_bits(a: np.ndarray) -> np.ndarray:
    """The bfloat16 bit patterns (uint16) of bf16-exact float32 values."""
    return (np.ascontiguousarray(a, np.float32).view(np.uint32) >> 16).astype(np.uint16)


@dataclasses.dataclass
class CorrWorkload:
    """Inputs of the correlation features of one window's patch graph."""
    fmap0: np.ndarray     # [F, H0, W0, D] float32, bf16-exact: first-level matching features
    fmap1: np.ndarray     # [F, H1, W1, D] float32, bf16-exact: second level (independent draw)
    gmap: np.ndarray      # [M, p*p, D] float32, bf16-exact: patch features
    coords: np.ndarray    # [E, p*p, 2] float32: reprojected pixels, first-level pixel units
    kk: np.ndarray        # [E] int32
    jj: np.ndarray        # [E] int32
    scale1: int           # second-level coordinate divisor

    @property
    def n_edges(self) -> int:
        return int(self.kk.shape[0])


def correlation_workload(n_frames: int, ppf: int, radius: int, *, seed: Sequence[int],
                         p: int = 3, dim: int = FEATURE_DIM, scale1: int = 4,
                         noise_px: float = 1.0, feature_hw=None) -> CorrWorkload:
    """Random N(0,1) features and a simulated patch graph: frame maps at 1/4
    of the 640x480 image, p x p patches of first-level pixels (spacing 1 =
    4 image pixels) around random centres, every patch joined to every frame
    within `radius` of its source frame.  Each patch pixel is back-projected
    at the patch's true depth (a fronto-parallel plane in its source frame),
    seen by the target camera and perturbed by N(0, noise_px) image pixels,
    so coordinates leave the map where the scene does.  `feature_hw` shrinks
    the first-level map (coordinates scale with it) for small cases."""
    w = make_window(n_frames, ppf, radius, seed=list(seed) + [77])
    rng = np.random.default_rng(list(seed) + [78])
    s0 = FEATURE_STRIDE
    H0, W0 = feature_hw if feature_hw is not None else (HEIGHT // s0, WIDTH // s0)
    H1, W1 = H0 // scale1, W0 // scale1
    fmap0 = bf16_exact(rng.normal(size=(n_frames, H0, W0, dim)).astype(np.float32))
    fmap1 = bf16_exact(rng.normal(size=(n_frames, H1, W1, dim)).astype(np.float32))
    M = w.n_patches
    gmap = bf16_exact(rng.normal(size=(M, p * p, dim)).astype(np.float32))
    sx, sy = WIDTH / W0, HEIGHT / H0              # image pixels per first-level pixel
    r = (p - 1) / 2.0
    offs = [((v - r) * sx, (u - r) * sy) for u in range(p) for v in range(p)]   # (dx, dy), row-major
    E = w.n_edges
    coords = np.empty((E, p * p, 2), np.float32)
    for q, (dx, dy) in enumerate(offs):
        px = np.stack([w.patches[:, 0] + dx, w.patches[:, 1] + dy, w.depth_gt], 1)
        Xw = scene_points(w.poses_gt, px, w.anchor, w.intrinsics)
        uv, _ = camera_observation(w.poses_gt, Xw[w.kk], w.jj, w.intrinsics)
        uv = uv + rng.normal(0.0, noise_px, uv.shape)
        coords[:, q, 0] = (uv[:, 0] / sx).astype(np.float32)
        coords[:, q, 1] = (uv[:, 1] / sy).astype(np.float32)
    return CorrWorkload(fmap0=fmap0, fmap1=fmap1, gmap=gmap, coords=coords,
                        kk=w.kk.copy(), jj=w.jj.copy(), scale1=scale1)


def method_scale_correlation(window_id: int = 0) -> CorrWorkload:
    """The 22-frame x 96-patch, radius-13 patch graph (39,552 edges, self-edges
    included) over 160 x 120 first-level and 40 x 30 second-level maps of 128
    channels, 3 x 3 patches."""
    return correlation_workload(22, 96, 13, seed=[2208, 5, window_id])


# ---------------------------------------------------------------- soft-aggregation workloads
HIDDEN_DIM = 384        # hidden state of an edge in the update operator


@dataclasses.dataclass
class AggWorkload:
    """Inputs of the soft aggregation over one window's patch graph."""
    x: np.ndarray          # [E, dim] float32, bf16-exact: hidden state of each edge
    kk: np.ndarray         # [E] int32
    jj: np.ndarray         # [E] int32
    anchor: np.ndarray     # [M] int32
    n_frames: int
    w: tuple               # 3 x [dim, dim] float32, bf16-exact: gate, value, output layers (out, in)
    b: tuple               # 3 x [dim] float32: their biases

    @property
    def n_edges(self) -> int:
        return int(self.kk.shape[0])


def aggregation_workload(n_frames: int, ppf: int, radius: int, *, seed: Sequence[int],
                         dim: int = HIDDEN_DIM) -> AggWorkload:
    """Random N(0,1) hidden states over the patch graph of a window (every
    patch joined to every frame within `radius` of its source frame) and
    random linear layers, weights N(0, 1/dim) and biases N(0, 0.01)."""
    rng = np.random.default_rng(list(seed))
    M = n_frames * ppf
    anchor = np.repeat(np.arange(n_frames, dtype=np.int32), ppf)
    kk_l, jj_l = [], []
    for k in range(M):
        i = int(anchor[k])
        for j in range(max(0, i - radius), min(n_frames - 1, i + radius) + 1):
            kk_l.append(k)
            jj_l.append(j)
    kk = np.asarray(kk_l, np.int32)
    jj = np.asarray(jj_l, np.int32)
    x = bf16_exact(rng.normal(size=(len(kk), dim)).astype(np.float32))
    w = tuple(bf16_exact((rng.normal(size=(dim, dim)) / np.sqrt(dim)).astype(np.float32)) for _ in range(3))
    b = tuple((rng.normal(size=dim) * 0.1).astype(np.float32) for _ in range(3))
    return AggWorkload(x=x, kk=kk, jj=jj, anchor=anchor, n_frames=n_frames, w=w, b=b)


def method_scale_aggregation(window_id: int = 0) -> AggWorkload:
    """The 22-frame x 96-patch, radius-13 patch graph (39,552 edges) with
    384-channel hidden states."""
    return aggregation_workload(22, 96, 13, seed=[2208, 10, window_id])


# ---------------------------------------------------------------- camera streams (sliding-window driver)
@dataclasses.dataclass
class Stream:
    """A synthetic camera stream for the sliding-window driver.

    The update operator, which revises the targets and weights of every edge,
    is replaced by a sensor table: for patch g (frame g // ppf) and frame f
    with |f - g // ppf| <= R, the target (the true projection plus noise) and
    the weight of edge (g, f)."""
    poses_gt: np.ndarray     # [T,7] true world->camera poses
    xy: np.ndarray           # [T, ppf, 2] patch centres of each frame (pixels)
    depth_gt: np.ndarray     # [T, ppf] true inverse depths
    table_t: np.ndarray      # [T*ppf, 2R+1, 2] targets of edge (g, g // ppf + o - R)
    table_w: np.ndarray      # [T*ppf, 2R+1, 2] weights (0 outside the stream and for hidden edges)
    init_poses: np.ndarray   # [2,7] poses of the first two frames (initialisation)
    init_depth: float        # inverse depth of the first frame's patches
    R: int
    intrinsics: np.ndarray   # [4]

    @property
    def n_frames(self) -> int:
        return int(self.poses_gt.shape[0])

    @property
    def ppf(self) -> int:
        return int(self.xy.shape[1])


def make_stream(n_frames: int, ppf: int, *, seed: Sequence[int], R: int = 40, outlier_frac: float = 0.1,
                fp32: bool = False) -> Stream:
    """Forward motion of 0.05 m per frame with a sideways component that
    alternates every 5 frames between slow (0.03 m) and fast (0.25 m) motion,
    0.5 degree rotation jitter; patches uniform over the image, inverse depth
    U[0.2, 1]; targets = true projection + N(0, 1 px), weights U[0.1, 1], 10%
    outliers (N(0, 20 px), weights U[0, 0.05]); edges whose true depth ratio is
    below HIDE_RATIO get weight 0 and the source pixel as target."""
    rng = np.random.default_rng(list(seed))
    intr = np.array([FX, FY, CX, CY])
    deg = np.pi / 180.0
    steps = [np.array([0.25 if (a // 5) % 2 else 0.03, 0.0, 0.05]) for a in range(n_frames)]
    centres = np.cumsum(np.stack(steps), 0) - steps[0]
    R_cw = [_rotvec_to_matrix(rng.normal(0.0, 0.5 * deg, 3)) for _ in range(n_frames)]
    poses_gt = np.stack([_camera(centres[a], R_cw[a]) for a in range(n_frames)])
    xy = np.stack([np.stack([rng.uniform(0, WIDTH, ppf), rng.uniform(0, HEIGHT, ppf)], -1)
                   for _ in range(n_frames)])
    depth_gt = rng.uniform(0.2, 1.0, (n_frames, ppf))
    G = n_frames * ppf
    anchor = np.repeat(np.arange(n_frames), ppf)
    patches = np.concatenate([xy.reshape(G, 2), depth_gt.reshape(G, 1)], 1)
    Xw = scene_points(poses_gt, patches, anchor, intr)
    table_t = np.zeros((G, 2 * R + 1, 2))
    table_w = np.zeros((G, 2 * R + 1, 2))
    for o in range(2 * R + 1):
        f = anchor + o - R
        ok = (f >= 0) & (f < n_frames)
        idx = np.nonzero(ok)[0]
        if len(idx) == 0:
            continue
        uv, depth = camera_observation(poses_gt, Xw[idx], f[idx], intr)
        t = uv + rng.normal(0.0, 1.0, uv.shape)
        w = rng.uniform(0.1, 1.0, uv.shape)
        out = rng.uniform(size=len(idx)) < outlier_frac
        t[out] = uv[out] + rng.normal(0.0, 20.0, (int(out.sum()), 2))
        w[out] = rng.uniform(0.0, 0.05, (int(out.sum()), 2))
        hidden = depth * depth_gt.reshape(G)[idx] < HIDE_RATIO
        t[hidden] = patches[idx[hidden], :2]
        w[hidden] = 0.0
        table_t[idx, o] = t
        table_w[idx, o] = w
    if fp32:
        table_t = table_t.astype(np.float32).astype(np.float64)
        table_w = table_w.astype(np.float32).astype(np.float64)
    return Stream(poses_gt=poses_gt, xy=xy, depth_gt=depth_gt, table_t=table_t, table_w=table_w,
                  init_poses=poses_gt[:2].copy(), init_depth=0.5, R=R, intrinsics=intr)
