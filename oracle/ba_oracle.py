"""FP64 CPU oracle of the bundle-adjustment layer of Deep Patch Visual Odometry
(Teed, Lipson, Deng, arXiv 2208.04726).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never calls it and
shares no code with it.

What it computes, plainly and slowly, in float64 on the CPU with PyTorch:

  * the reprojection of a patch centre from its source frame i into frame j,
    x' ~ K T_j T_i^{-1} K^{-1} (x, y, 1, d), divided by the third element
    (Sec. 3 "Preliminaries", Eq. 2 and the 4x4 calibration matrix Eq. 3);
  * the weighted least-squares objective over the patch-graph edges,
    sum_(k,j) || omega_ij(T, P_k) - target_kj ||^2_Sigma_kj  (Sec. 3.1
    "Differentiable Bundle Adjustment", Eq. 6), with the confidence Sigma read
    as a diagonal weight (higher = more trust);
  * Gauss-Newton iterations on that objective over the free poses and every
    patch's inverse depth, pixel coordinates held constant (Sec. 3.1), a fixed
    number of iterations (two in the paper, Sec. 3.1 and Sec. 3.3
    "Optimization"), the poses outside the optimisation window fixed
    (Sec. 3.3), and damping 1e-4 (Appendix "Bundle Adjustment Layer").

Each Gauss-Newton step is written as its plain definition: build the damped
normal equations H = sum_e J_e^T W_e J_e + lambda I, g = sum_e J_e^T W_e r_e
over all free unknowns as ONE dense matrix and solve H delta = -g with a library
solver.  The Schur complement the paper uses is only a faster route to the same
delta, so it does not appear here.  Gradients of a loss of the solved state
with respect to targets and weights are plain autograd through these steps
(the paper back-propagates through the Gauss-Newton iterations, Sec. 3.1).

Readings taken where the paper is silent (each is listed in the design notes):
  * poses are world->camera, stored (tx,ty,tz,qx,qy,qz,qw), unit Hamilton
    quaternion with the scalar last;
  * tangent xi = (rho, phi), translation first; retraction T <- Exp(xi) T
    (left); Exp from Rodrigues' formula with its V matrix;
  * an edge is active iff j != source frame and the projected homogeneous
    depth Z > z_min (0.1); inactive edges contribute nothing;
  * lambda is added to the diagonal of every free unknown (poses and depths);
  * no clamping of inverse depth, no line search, no early exit.
"""
from __future__ import annotations

from typing import Dict, Optional

import numpy as np
import torch

DT = torch.float64
SMALL_ANGLE = 1e-2   # below this rotation angle the series forms are used


# --------------------------------------------------------------- rotations
def hat(v: torch.Tensor) -> torch.Tensor:
    """[...,3] -> [...,3,3] cross-product matrix: hat(a) @ b = a x b."""
    z = torch.zeros_like(v[..., 0])
    return torch.stack([
        torch.stack([z, -v[..., 2], v[..., 1]], -1),
        torch.stack([v[..., 2], z, -v[..., 0]], -1),
        torch.stack([-v[..., 1], v[..., 0], z], -1)], -2)


def quat_to_rot(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrix of a unit quaternion (x, y, z, w)."""
    x, y, z, w = q.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        torch.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        torch.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1)], -2)


def quat_mul(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """Hamilton product a (x) b of (x, y, z, w) quaternions."""
    av, aw = a[..., :3], a[..., 3:]
    bv, bw = b[..., :3], b[..., 3:]
    v = aw * bv + bw * av + torch.cross(av, bv, dim=-1)
    w = aw * bw - (av * bv).sum(-1, keepdim=True)
    return torch.cat([v, w], -1)


def _angle_terms(phi: torch.Tensor):
    """theta^2 and a safe theta (1 where theta is small, so that no branch of
    a torch.where ever produces a non-finite value or gradient)."""
    th2 = (phi * phi).sum(-1)
    small = th2 < SMALL_ANGLE ** 2
    th = torch.sqrt(torch.where(small, torch.ones_like(th2), th2))
    return th2, th, small


def so3_exp_quat(phi: torch.Tensor) -> torch.Tensor:
    """Unit quaternion of the rotation vector phi: (sin(t/2) phi/t, cos(t/2))."""
    th2, th, small = _angle_terms(phi)
    s_series = 0.5 - th2 / 48.0 + th2 * th2 / 3840.0
    c_series = 1.0 - th2 / 8.0 + th2 * th2 / 384.0
    s = torch.where(small, s_series, torch.sin(th / 2) / th)
    c = torch.where(small, c_series, torch.cos(th / 2))
    return torch.cat([s[..., None] * phi, c[..., None]], -1)


def so3_exp(phi: torch.Tensor) -> torch.Tensor:
    """Rodrigues: R = I + A hat(phi) + B hat(phi)^2."""
    th2, th, small = _angle_terms(phi)
    A = torch.where(small, 1 - th2 / 6 + th2 * th2 / 120 - th2 ** 3 / 5040,
                    torch.sin(th) / th)
    B = torch.where(small, 0.5 - th2 / 24 + th2 * th2 / 720 - th2 ** 3 / 40320,
                    (1 - torch.cos(th)) / (th * th))
    K = hat(phi)
    I = torch.eye(3, dtype=phi.dtype).expand(K.shape)
    return I + A[..., None, None] * K + B[..., None, None] * (K @ K)


def se3_exp(xi: torch.Tensor):
    """Exp of xi = (rho, phi): rotation R(phi) and translation V(phi) rho with
    V = I + B hat(phi) + C hat(phi)^2."""
    rho, phi = xi[..., :3], xi[..., 3:]
    th2, th, small = _angle_terms(phi)
    B = torch.where(small, 0.5 - th2 / 24 + th2 * th2 / 720 - th2 ** 3 / 40320,
                    (1 - torch.cos(th)) / (th * th))
    C = torch.where(small, 1.0 / 6 - th2 / 120 + th2 * th2 / 5040 - th2 ** 3 / 362880,
                    (th - torch.sin(th)) / (th * th * th))
    K = hat(phi)
    I = torch.eye(3, dtype=xi.dtype).expand(K.shape)
    V = I + B[..., None, None] * K + C[..., None, None] * (K @ K)
    return so3_exp(phi), (V @ rho[..., None])[..., 0]


def retract(pose: torch.Tensor, xi: torch.Tensor) -> torch.Tensor:
    """Left retraction T <- Exp(xi) T on 7-vector poses; quaternion renormalised."""
    R, t = se3_exp(xi)
    t_new = (R @ pose[..., :3, None])[..., 0] + t
    q_new = quat_mul(so3_exp_quat(xi[..., 3:]), pose[..., 3:])
    q_new = q_new / torch.linalg.norm(q_new, dim=-1, keepdim=True)
    return torch.cat([t_new, q_new], -1)


def adjoint(R: torch.Tensor, t: torch.Tensor) -> torch.Tensor:
    """6x6 adjoint of (R, t) for the (rho, phi) tangent: [[R, hat(t) R], [0, R]]."""
    top = torch.cat([R, hat(t) @ R], -1)
    bot = torch.cat([torch.zeros_like(R), R], -1)
    return torch.cat([top, bot], -2)


# --------------------------------------------------------------- edge model
def relative_poses(poses: torch.Tensor, ii: torch.Tensor, jj: torch.Tensor):
    """T_ji = T_j T_i^{-1} for each edge: R_ji = R_j R_i^T, t_ji = t_j - R_ji t_i."""
    Ri = quat_to_rot(poses[ii, 3:])
    Rj = quat_to_rot(poses[jj, 3:])
    R = Rj @ Ri.transpose(-1, -2)
    t = poses[jj, :3] - (R @ poses[ii, :3, None])[..., 0]
    return R, t


def edge_linearization(poses, depth, patches_xy, anchor, kk, jj, targets, intr,
                       z_min: float = 0.1):
    """Residuals and Jacobians of every edge (Eq. 2, Eq. 3, Eq. 6).

    Returns dict with r [E,2], Ji [E,2,6], Jj [E,2,6], Jd [E,2], active [E]
    (bool), Z [E].  Inactive edges have r = 0 and zero Jacobians."""
    fx, fy, cx, cy = intr
    ii = anchor[kk]
    R, t = relative_poses(poses, ii, jj)
    d = depth[kk]
    h = torch.stack([(patches_xy[kk, 0] - cx) / fx, (patches_xy[kk, 1] - cy) / fy,
                     torch.ones_like(d)], -1)
    p = (R @ h[..., None])[..., 0] + t * d[:, None]          # K^-1-free part of Eq. 2
    Z = p[:, 2]
    active = (ii != jj) & (Z > z_min)
    Zs = torch.where(active, Z, torch.ones_like(Z))
    X, Y = p[:, 0], p[:, 1]
    pi = torch.stack([fx * X / Zs + cx, fy * Y / Zs + cy], -1)   # divide by 3rd element
    r = torch.where(active[:, None], pi - targets, torch.zeros_like(pi))
    zero = torch.zeros_like(Zs)
    Pi = torch.stack([torch.stack([fx / Zs, zero, -fx * X / (Zs * Zs)], -1),
                      torch.stack([zero, fy / Zs, -fy * Y / (Zs * Zs)], -1)], -2)  # d pi / d p
    # d p / d(left perturbation of T_j) = [d I | -hat(p)]
    dp_dxj = torch.cat([d[:, None, None] * torch.eye(3, dtype=DT).expand(len(d), 3, 3),
                        -hat(p)], -1)
    Jj = Pi @ dp_dxj
    Ji = -Jj @ adjoint(R, t)
    Jd = (Pi @ t[..., None])[..., 0]
    m = active[:, None, None].to(DT)
    return dict(r=r, Ji=Ji * m, Jj=Jj * m, Jd=Jd * m[..., 0], active=active, Z=Z)


# --------------------------------------------------------------- GN step
def unknown_layout(n_frames: int, n_patches: int, n_fixed: int):
    """Column of each unknown: pose a >= n_fixed -> 6 (a - n_fixed) .. +5,
    depth k -> 6 (n_frames - n_fixed) + k.  Fixed poses map to a sink column
    `n` that is dropped."""
    n_pose = 6 * max(n_frames - n_fixed, 0)
    n = n_pose + n_patches
    pose_col = torch.full((n_frames, 6), n, dtype=torch.long)
    for a in range(n_fixed, n_frames):
        pose_col[a] = torch.arange(6 * (a - n_fixed), 6 * (a - n_fixed) + 6)
    depth_col = n_pose + torch.arange(n_patches)
    return n, n_pose, pose_col, depth_col


def normal_equations(poses, depth, P: Dict, lam: float, z_min: float = 0.1):
    """Dense damped normal equations over all free unknowns:
    H = sum_e J_e^T W_e J_e + lam I,  g = sum_e J_e^T W_e r_e."""
    lin = edge_linearization(poses, depth, P["patches_xy"], P["anchor"], P["kk"],
                             P["jj"], P["targets"], P["intr"], z_min)
    N, M = poses.shape[0], depth.shape[0]
    n, n_pose, pose_col, depth_col = unknown_layout(N, M, P["n_fixed"])
    ii = P["anchor"][P["kk"]]
    J = torch.cat([lin["Ji"], lin["Jj"], lin["Jd"][..., None]], -1)          # [E,2,13]
    cols = torch.cat([pose_col[ii], pose_col[P["jj"]], depth_col[P["kk"]][:, None]], -1)  # [E,13]
    Wt = P["weights"]
    JtW = J.transpose(-1, -2) * Wt[:, None, :]                              # [E,13,2]
    He = JtW @ J                                                             # [E,13,13]
    ge = (JtW @ lin["r"][..., None])[..., 0]                                 # [E,13]
    H = torch.zeros((n + 1, n + 1), dtype=DT)
    g = torch.zeros(n + 1, dtype=DT)
    rows = cols[:, :, None].expand(-1, 13, 13)
    colm = cols[:, None, :].expand(-1, 13, 13)
    H = H.index_put((rows.reshape(-1), colm.reshape(-1)), He.reshape(-1), accumulate=True)
    g = g.index_put((cols.reshape(-1),), ge.reshape(-1), accumulate=True)
    H = H[:n, :n] + lam * torch.eye(n, dtype=DT)
    return H, g[:n], lin, (n_pose, pose_col, depth_col)


def gn_step(poses, depth, P: Dict, lam: float = 1e-4, z_min: float = 0.1):
    """One Gauss-Newton step: delta = -H^{-1} g, then T_a <- Exp(dxi_a) T_a for
    free poses and d_k <- d_k + dd_k."""
    H, g, lin, (n_pose, pose_col, depth_col) = normal_equations(poses, depth, P, lam, z_min)
    delta = -torch.linalg.solve(H, g)
    nf = P["n_fixed"]
    N = poses.shape[0]
    if N > nf:
        dxi = delta[:n_pose].reshape(N - nf, 6)
        new_free = retract(poses[nf:], dxi)
        poses = torch.cat([poses[:nf], new_free], 0)
    depth = depth + delta[n_pose:]
    return poses, depth, dict(H=H, g=g, delta=delta, lin=lin)


def to_problem(w, dtype=DT) -> Dict:
    """Torch tensors of a synth.Window-like object (fields poses, patches,
    anchor, kk, jj, targets, weights, intrinsics, n_fixed)."""
    return dict(
        poses=torch.as_tensor(np.asarray(w.poses), dtype=dtype),
        depth=torch.as_tensor(np.asarray(w.patches)[:, 2], dtype=dtype),
        patches_xy=torch.as_tensor(np.asarray(w.patches)[:, :2], dtype=dtype),
        anchor=torch.as_tensor(np.asarray(w.anchor), dtype=torch.long),
        kk=torch.as_tensor(np.asarray(w.kk), dtype=torch.long),
        jj=torch.as_tensor(np.asarray(w.jj), dtype=torch.long),
        targets=torch.as_tensor(np.asarray(w.targets), dtype=dtype),
        weights=torch.as_tensor(np.asarray(w.weights), dtype=dtype),
        intr=[float(v) for v in np.asarray(w.intrinsics)],
        n_fixed=int(w.n_fixed))


def solve(w, iterations: int = 2, lam: float = 1e-4, z_min: float = 0.1,
          P: Optional[Dict] = None):
    """K Gauss-Newton steps from the window's initial state.
    Returns (poses [N,7] numpy, inverse depths [M] numpy)."""
    P = to_problem(w) if P is None else P
    with torch.no_grad():
        poses, depth = P["poses"], P["depth"]
        for _ in range(iterations):
            poses, depth, _ = gn_step(poses, depth, P, lam, z_min)
    return poses.numpy(), depth.numpy()


def solve_torch(P: Dict, iterations: int = 2, lam: float = 1e-4, z_min: float = 0.1):
    """K steps on torch tensors, differentiable in P['targets'], P['weights']."""
    poses, depth = P["poses"], P["depth"]
    for _ in range(iterations):
        poses, depth, _ = gn_step(poses, depth, P, lam, z_min)
    return poses, depth


def camera_centres(poses: torch.Tensor) -> torch.Tensor:
    """c = -R^T t for world->camera poses."""
    R = quat_to_rot(poses[..., 3:])
    return -(R.transpose(-1, -2) @ poses[..., :3, None])[..., 0]


def translation_loss_grad(w, iterations: int = 2, lam: float = 1e-4, z_min: float = 0.1):
    """L = sum over free frames of ||c_a - c_a^gt||^2 after K steps, and its
    gradient with respect to targets [E,2] and weights [E,2]."""
    P = to_problem(w)
    P["targets"].requires_grad_(True)
    P["weights"].requires_grad_(True)
    poses, depth = solve_torch(P, iterations, lam, z_min)
    gt = torch.as_tensor(np.asarray(w.poses_gt), dtype=DT)
    nf = P["n_fixed"]
    L = ((camera_centres(poses[nf:]) - camera_centres(gt[nf:])) ** 2).sum()
    gy, gw = torch.autograd.grad(L, (P["targets"], P["weights"]))
    return float(L.detach()), gy.numpy(), gw.numpy()


def cotangent_grad(w, grad_poses: np.ndarray, grad_depth: np.ndarray,
                   iterations: int = 2, lam: float = 1e-4, z_min: float = 0.1):
    """Vector-Jacobian product of the K-step map: given cotangents of the
    output pose 7-vectors [N,7] and inverse depths [M], return the gradient
    with respect to targets [E,2] and weights [E,2]."""
    P = to_problem(w)
    P["targets"].requires_grad_(True)
    P["weights"].requires_grad_(True)
    poses, depth = solve_torch(P, iterations, lam, z_min)
    L = (poses * torch.as_tensor(grad_poses, dtype=DT)).sum() + \
        (depth * torch.as_tensor(grad_depth, dtype=DT)).sum()
    gy, gw = torch.autograd.grad(L, (P["targets"], P["weights"]))
    return gy.numpy(), gw.numpy()


def reduced_system(w, poses=None, depth=None, lam: float = 1e-4, z_min: float = 0.1):
    """The damped normal equations at a state, split into the pose block, the
    pose-depth block and the depth diagonal; and the depth-eliminated pose
    system S = Hpp - Hpd Hdd^{-1} Hdp, s = gp - Hpd Hdd^{-1} gd (the Schur
    complement the paper names, written as its definition for comparison of
    intermediate results)."""
    P = to_problem(w)
    poses = P["poses"] if poses is None else torch.as_tensor(poses, dtype=DT)
    depth = P["depth"] if depth is None else torch.as_tensor(depth, dtype=DT)
    with torch.no_grad():
        H, g, lin, (n_pose, _, _) = normal_equations(poses, depth, P, lam, z_min)
        Hpp, Hpd, Hdd = H[:n_pose, :n_pose], H[:n_pose, n_pose:], H[n_pose:, n_pose:]
        gp, gd = g[:n_pose], g[n_pose:]
        Hdd_inv = torch.linalg.inv(Hdd)
        S = Hpp - Hpd @ Hdd_inv @ Hpd.T
        s = gp - Hpd @ Hdd_inv @ gd
    return S.numpy(), s.numpy()


# --------------------------------------------------------------- large windows
def normal_blocks(poses, depth, P: Dict, lam: float, z_min: float = 0.1):
    """The damped normal equations of `normal_equations`, kept in three blocks
    so that windows with tens of thousands of depths fit in memory:
      Hpp [n_pose, n_pose] dense,  Hpd [n_pose, M] dense,  hdd [M] (the depth
      block is diagonal: every edge involves exactly one depth),  gp, gd.
    Each block is the same sum over edges of J_e^T W_e J_e (and J_e^T W_e r_e)
    restricted to its unknowns; lam is added to every free diagonal."""
    lin = edge_linearization(poses, depth, P["patches_xy"], P["anchor"], P["kk"],
                             P["jj"], P["targets"], P["intr"], z_min)
    N, M = poses.shape[0], depth.shape[0]
    nf = P["n_fixed"]
    kk, jj = P["kk"], P["jj"]
    ii = P["anchor"][kk]
    W = P["weights"]
    Ji, Jj, Jd, r = lin["Ji"], lin["Jj"], lin["Jd"], lin["r"]
    JiW = Ji.transpose(-1, -2) * W[:, None, :]        # [E,6,2]
    JjW = Jj.transpose(-1, -2) * W[:, None, :]
    # pose-pose: blocks (i,i), (i,j), (j,i), (j,j) of every edge, summed per frame pair
    Bpair = torch.zeros((N * N, 6, 6), dtype=DT)
    Bpair.index_add_(0, ii * N + ii, JiW @ Ji)
    Bpair.index_add_(0, ii * N + jj, JiW @ Jj)
    Bpair.index_add_(0, jj * N + ii, JjW @ Ji)
    Bpair.index_add_(0, jj * N + jj, JjW @ Jj)
    Bfull = Bpair.reshape(N, N, 6, 6).permute(0, 2, 1, 3).reshape(6 * N, 6 * N)
    gfull = torch.zeros(6 * N, dtype=DT)
    gfull.index_add_(0, (6 * ii[:, None] + torch.arange(6)).reshape(-1), (JiW @ r[..., None]).reshape(-1))
    gfull.index_add_(0, (6 * jj[:, None] + torch.arange(6)).reshape(-1), (JjW @ r[..., None]).reshape(-1))
    # pose-depth: J_a^T W J_d into (pose a, patch k)
    Hpd_full = torch.zeros((6 * N, M), dtype=DT)
    rows_i = (6 * ii[:, None] + torch.arange(6)).reshape(-1)
    rows_j = (6 * jj[:, None] + torch.arange(6)).reshape(-1)
    colk = kk[:, None].expand(-1, 6).reshape(-1)
    Hpd_full.index_put_((rows_i, colk), (JiW @ Jd[..., None]).reshape(-1), accumulate=True)
    Hpd_full.index_put_((rows_j, colk), (JjW @ Jd[..., None]).reshape(-1), accumulate=True)
    # depth diagonal and depth gradient
    hdd = torch.zeros(M, dtype=DT).index_add_(0, kk, (W * Jd * Jd).sum(-1)) + lam
    gd = torch.zeros(M, dtype=DT).index_add_(0, kk, (W * Jd * r).sum(-1))
    fr = slice(6 * nf, 6 * N)
    n_pose = 6 * (N - nf)
    Hpp = Bfull[fr, fr] + lam * torch.eye(n_pose, dtype=DT)
    return Hpp, Hpd_full[fr], hdd, gfull[fr], gd, lin


def gn_step_schur(poses, depth, P: Dict, lam: float = 1e-4, z_min: float = 0.1):
    """The Gauss-Newton step of `gn_step`, with the depths eliminated first
    (the Schur complement of Sec. 3.1, an exact identity since the depth block
    is diagonal):
      S = Hpp - Hpd diag(hdd)^-1 Hpd^T,   s = gp - Hpd (gd / hdd),
      dxi = -S^-1 s (library Cholesky),   dd = -(gd + Hpd^T dxi) / hdd."""
    Hpp, Hpd, hdd, gp, gd, lin = normal_blocks(poses, depth, P, lam, z_min)
    S = Hpp - (Hpd / hdd) @ Hpd.T
    s = gp - Hpd @ (gd / hdd)
    nf = P["n_fixed"]
    N = poses.shape[0]
    if S.shape[0] > 0:
        L = torch.linalg.cholesky(S)
        dxi = -torch.cholesky_solve(s[:, None], L)[:, 0]
    else:
        dxi = torch.zeros(0, dtype=DT)
    dd = -(gd + Hpd.T @ dxi) / hdd
    if N > nf:
        poses = torch.cat([poses[:nf], retract(poses[nf:], dxi.reshape(N - nf, 6))], 0)
    return poses, depth + dd, dict(S=S, s=s)


def solve_schur(w, iterations: int = 2, lam: float = 1e-4, z_min: float = 0.1):
    """K steps of `gn_step_schur` (for windows too large for the dense H).
    Returns (poses [N,7] numpy, inverse depths [M] numpy)."""
    P = to_problem(w)
    with torch.no_grad():
        poses, depth = P["poses"], P["depth"]
        for _ in range(iterations):
            poses, depth, _ = gn_step_schur(poses, depth, P, lam, z_min)
    return poses.numpy(), depth.numpy()
