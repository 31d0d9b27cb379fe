"""Tolerance aid for the FP32-assembly parity tests (not part of the oracle).

`solve_schur_rounded` runs the oracle's block-eliminated Gauss-Newton step with
its reduced system (S, s) rounded once to FP32 before the FP64 solve: the
result of a pipeline whose assembly is exact up to one rounding of every entry
of the reduced system.  How far that moves the solution measures how strongly
a window's conditioning amplifies assembly rounding; the FP32 tests scale
their bounds with it.  It composes the oracle's public pieces (the normal
blocks, the retraction) and adds only the rounding.
"""
import numpy as np
import torch

from oracle import ba_oracle as O


def solve_schur_rounded(w, iterations=2, dtype=torch.float32, lam=1e-4, z_min=0.1):
    P = O.to_problem(w)
    poses, depth = P["poses"], P["depth"]
    nf, N = P["n_fixed"], poses.shape[0]
    with torch.no_grad():
        for _ in range(iterations):
            Hpp, Hpd, hdd, gp, gd, _ = O.normal_blocks(poses, depth, P, lam, z_min)
            S = (Hpp - (Hpd / hdd) @ Hpd.T).to(dtype).to(O.DT)
            s = (gp - Hpd @ (gd / hdd)).to(dtype).to(O.DT)
            if S.shape[0] > 0:
                dxi = -torch.cholesky_solve(s[:, None], torch.linalg.cholesky(S))[:, 0]
            else:
                dxi = torch.zeros(0, dtype=O.DT)
            depth = depth - (gd + Hpd.T @ dxi) / hdd
            if N > nf:
                poses = torch.cat([poses[:nf], O.retract(poses[nf:], dxi.reshape(N - nf, 6))], 0)
    return poses.numpy(), depth.numpy()


def translation_loss_grad_rounded(w, iterations=2, dtype=torch.float32, lam=1e-4, z_min=0.1):
    """L = sum of squared free camera-centre errors after `iterations` steps of
    the block-eliminated solve with (S, s) rounded to `dtype` as in
    `solve_schur_rounded`, and its gradient with respect to targets and
    weights (the rounding passes the gradient through unchanged).  How far
    this gradient lies from the oracle's exact one measures how strongly the
    loss amplifies assembly rounding."""
    P = O.to_problem(w)
    P["targets"].requires_grad_(True)
    P["weights"].requires_grad_(True)
    poses, depth = P["poses"], P["depth"]
    nf, N = P["n_fixed"], poses.shape[0]
    for _ in range(iterations):
        Hpp, Hpd, hdd, gp, gd, _ = O.normal_blocks(poses, depth, P, lam, z_min)
        S = (Hpp - (Hpd / hdd) @ Hpd.T).to(dtype).to(O.DT)
        s = (gp - Hpd @ (gd / hdd)).to(dtype).to(O.DT)
        dxi = -torch.cholesky_solve(s[:, None], torch.linalg.cholesky(S))[:, 0]
        depth = depth - (gd + Hpd.T @ dxi) / hdd
        poses = torch.cat([poses[:nf], O.retract(poses[nf:], dxi.reshape(N - nf, 6))], 0)
    gt = torch.as_tensor(np.asarray(w.poses_gt), dtype=O.DT)
    L = ((O.camera_centres(poses[nf:]) - O.camera_centres(gt[nf:])) ** 2).sum()
    gy, gw = torch.autograd.grad(L, (P["targets"], P["weights"]))
    return float(L.detach()), gy.numpy(), gw.numpy()


def cotangent_grad_rounded(w, grad_poses, grad_depth, iterations=2, dtype=torch.float32, lam=1e-4, z_min=0.1):
    """The oracle's vector-Jacobian product (cotangents of the output pose
    7-vectors and inverse depths) through `iterations` steps of the
    block-eliminated solve with (S, s) rounded to `dtype` as in
    `solve_schur_rounded` (the rounding passes the gradient through
    unchanged): how far it lies from the exact product measures how strongly
    the map amplifies assembly rounding."""
    P = O.to_problem(w)
    P["targets"].requires_grad_(True)
    P["weights"].requires_grad_(True)
    poses, depth = P["poses"], P["depth"]
    nf, N = P["n_fixed"], poses.shape[0]
    for _ in range(iterations):
        Hpp, Hpd, hdd, gp, gd, _ = O.normal_blocks(poses, depth, P, lam, z_min)
        S = Hpp - (Hpd / hdd) @ Hpd.T
        s = gp - Hpd @ (gd / hdd)
        S = S + (S.detach().to(dtype).to(O.DT) - S.detach())
        s = s + (s.detach().to(dtype).to(O.DT) - s.detach())
        dxi = -torch.cholesky_solve(s[:, None], torch.linalg.cholesky(S))[:, 0]
        depth = depth - (gd + Hpd.T @ dxi) / hdd
        poses = torch.cat([poses[:nf], O.retract(poses[nf:], dxi.reshape(N - nf, 6))], 0)
    L = (poses * torch.as_tensor(grad_poses, dtype=O.DT)).sum() + \
        (depth * torch.as_tensor(grad_depth, dtype=O.DT)).sum()
    gy, gw = torch.autograd.grad(L, (P["targets"], P["weights"]))
    return gy.numpy(), gw.numpy()


# Probabilistic rounding-error model (Higham and Mary, "A new approach to
# probabilistic rounding error analysis", SIAM J. Sci. Comput. 2019): a sum of
# m terms formed in a precision with unit roundoff u is, with high
# probability, within about sqrt(m) u of the summed magnitudes, where the
# worst case is m u.  The FP32 assembly forms each entry of a source frame's
# contribution to (S, s) as an FP32 sum over the frame's patches before the
# FP64 fold, so against one rounding of the final (S, s) it carries about
# sqrt(patches per source frame) times the perturbation.
def fp32_assembly_factor(w):
    """sqrt of the largest number of patches any source frame holds."""
    counts = np.bincount(np.asarray(w.anchor), minlength=w.n_frames)
    return float(np.sqrt(max(int(counts.max()), 1)))


# Depth sensitivity: how many times its relative input perturbation a patch's
# inverse depth moves.  Patches with kappa below KAPPA_WELL are held to the
# fixed relative bound; the few above it (weakly observed, outlier-dominated
# patches whose depth the Gauss-Newton steps move far) amplify every rounding
# by orders of magnitude and are reported with a sanity bound.
KAPPA_WELL = 100.0


def depth_sensitivity(w, iterations=2, eps=2.0 ** -18, seed=5):
    """Per patch: |d(perturbed) - d| / |d| / eps, where every target and
    weight is scaled by an independent random factor in [1 - eps, 1 + eps]
    (eps = 2^-18, about 32 FP32 ulps)."""
    _, d0 = O.solve_schur(w, iterations=iterations)
    rng = np.random.default_rng(seed)
    w2 = w.copy()
    w2.targets = w.targets * (1 + eps * rng.uniform(-1, 1, w.targets.shape))
    w2.weights = w.weights * (1 + eps * rng.uniform(-1, 1, w.weights.shape))
    _, d1 = O.solve_schur(w2, iterations=iterations)
    return np.abs(d1 - d0) / np.abs(d0) / eps


def check_depths(d_gpu, d_ref, kappa, bound=1e-3, rest_bound=5e-2, label="", rest_frac=1e-3):
    """Asserts the fixed relative `bound` on every patch with kappa <
    KAPPA_WELL; prints the count and worst case of the others, which must be
    at most `rest_frac` of the patches (at least 2) and within `rest_bound`."""
    rel = np.abs(d_gpu - d_ref) / np.abs(d_ref)
    well = kappa < KAPPA_WELL
    worst = float(rel[well].max()) if well.any() else 0.0
    msg = f"{label} depth: {int(well.sum())} patches with kappa < {KAPPA_WELL:g}, max rel {worst:.2e}"
    rest = np.nonzero(~well)[0]
    if len(rest):
        k = rest[np.argmax(rel[rest])]
        msg += f"; {len(rest)} others, worst {rel[k]:.2e} at patch {k} (kappa {kappa[k]:.0f})"
    print(msg)
    assert worst <= bound, msg
    assert len(rest) <= max(2, int(rest_frac * len(rel))), msg
    assert len(rest) == 0 or rel[rest].max() <= rest_bound, msg
