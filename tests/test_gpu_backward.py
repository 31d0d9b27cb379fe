"""Adjoint of the GPU solve (ba_backward through the C ABI) against the FP64
oracle's autograd and against FP64 central differences."""
import numpy as np
import pytest
import torch

from oracle import ba_oracle as O
from paper_2208_04726_amd import synth
from tests.gpu_util import need_gpu

pytestmark = pytest.mark.gpu


def gpu_vjp(w, gp, gd, precision):
    from paper_2208_04726_amd.solver import Solver, make_batch, capacities_for
    s = Solver(precision=precision, **capacities_for([w]))
    b = make_batch([w], precision)
    gt, gw = s.backward(b, torch.as_tensor(gp), torch.as_tensor(gd))
    torch.cuda.synchronize()
    st = s.status()
    s.close()
    return gt.double().cpu().numpy(), gw.double().cpu().numpy(), st


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("win", [0, 1])
def test_vjp_fp64_matches_oracle_autograd(win):
    need_gpu()
    w = synth.plain_fp64_window(win)
    rng = np.random.default_rng(win)
    gp = rng.normal(size=(w.n_frames, 7))
    gd = rng.normal(size=w.n_patches)
    gy_ref, gw_ref = O.cotangent_grad(w, gp, gd)
    gy, gwt, st = gpu_vjp(w, gp, gd, "fp64")
    assert st[0] == 0
    print("fp64 vjp rel err targets", rel_err(gy, gy_ref), "weights", rel_err(gwt, gw_ref))
    assert rel_err(gy, gy_ref) < 1e-8
    assert rel_err(gwt, gw_ref) < 1e-8


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("fp32", 1e-3)])
def test_vjp_method_scale_matches_oracle(precision, tol):
    """Fixed random cotangents on the 22 x 96 window: isolates the adjoint
    (FP32 path: FP32 linearisation, FP64 solves and adjoint arithmetic)."""
    need_gpu()
    w = synth.method_scale_window(2)
    rng = np.random.default_rng(7)
    gp = rng.normal(size=(w.n_frames, 7))
    gd = rng.normal(size=w.n_patches)
    gy_ref, gw_ref = O.cotangent_grad(w, gp, gd)
    gy, gwt, st = gpu_vjp(w, gp, gd, precision)
    assert st[0] == 0
    print(precision, "method-scale vjp rel err targets", rel_err(gy, gy_ref), "weights", rel_err(gwt, gw_ref))
    assert rel_err(gy, gy_ref) < tol
    assert rel_err(gwt, gw_ref) < tol


def _fd_floor(magnitude, h):
    """Absolute error floor of an FP64 central difference of a function whose
    terms sum to `magnitude` in absolute value (both evaluations rounded, over
    the step 2h, margin 10)."""
    return 10.0 * np.finfo(np.float64).eps * magnitude / h


@pytest.mark.parametrize("precision,win", [("fp64", 0), ("fp32", 0), ("fp32", 2), ("fp32", 3)])
def test_translation_loss_grad_method_scale(precision, win):
    """End to end through BAFunction on 22 x 96 windows: L = sum of squared
    free camera-centre errors, gradient with respect to targets and weights
    against the oracle's autograd.  FP64 assembly: 1e-8.  FP32 assembly: the
    loss sits near its minimum (centre errors of a few mm), so its gradient
    moves with the forward state; the bound is the change the oracle's own
    gradient shows when its reduced system is rounded once to FP32, times the
    summation factor sqrt(patches per source frame), and at least 1e-4."""
    need_gpu()
    from paper_2208_04726_amd.solver import BAFunction, Solver, make_batch, capacities_for
    from tests.rounding import fp32_assembly_factor, translation_loss_grad_rounded
    w = synth.method_scale_window(win)
    L_ref, gy_ref, gw_ref = O.translation_loss_grad(w)
    s = Solver(precision=precision, **capacities_for([w]))
    b = make_batch([w], precision)
    tg = b.targets.clone().requires_grad_(True)
    wt = b.weights.clone().requires_grad_(True)
    poses, depth = BAFunction.apply(tg, wt, s, b)
    q = poses[:, 3:]
    x, y, z, qw = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    Rm = torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * qw), 2 * (x * z + y * qw)], -1),
        torch.stack([2 * (x * y + z * qw), 1 - 2 * (x * x + z * z), 2 * (y * z - x * qw)], -1),
        torch.stack([2 * (x * z - y * qw), 2 * (y * z + x * qw), 1 - 2 * (x * x + y * y)], -1)], -2)
    c = -(Rm.transpose(-1, -2) @ poses[:, :3, None])[..., 0]
    gt_c = torch.as_tensor(synth.camera_centres(w.poses_gt), device=c.device)
    L = ((c[w.n_fixed:] - gt_c[w.n_fixed:]) ** 2).sum()
    L.backward()
    torch.cuda.synchronize()
    gy = tg.grad.double().cpu().numpy()
    gwt = wt.grad.double().cpu().numpy()
    eg, ew = rel_err(gy, gy_ref), rel_err(gwt, gw_ref)
    Lv = float(L.detach())
    if precision == "fp64":
        print(f"fp64 window {win}: L {Lv:.6e} (oracle {L_ref:.6e}), gradient rel err targets {eg:.2e} weights {ew:.2e}")
        assert abs(Lv - L_ref) < 1e-8 * L_ref
        assert eg < 1e-8 and ew < 1e-8
        return
    _, gy32, gw32 = translation_loss_grad_rounded(w)
    f = fp32_assembly_factor(w)
    tol_y = max(1e-4, f * rel_err(gy32, gy_ref))
    tol_w = max(1e-4, f * rel_err(gw32, gw_ref))
    print(f"fp32 window {win}: L {Lv:.6e} (oracle {L_ref:.6e}), gradient rel err targets {eg:.2e} "
          f"(bound {tol_y:.1e}) weights {ew:.2e} (bound {tol_w:.1e})")
    assert eg < tol_y and ew < tol_w


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_vjp_subwindow_vs_central_differences(precision):
    """ba_backward on the 6 x 8 sub-window (targets and weights FP32-exact)
    against FP64 central differences (step 1e-6) of f = <poses_out, g_p> +
    <depth_out, g_d> through the oracle, entry by entry over every active edge
    and both coordinates.  FP64 assembly: relative 1e-4 above the rounding
    floor of the difference quotient.  FP32 assembly: its iterates carry the
    FP32 forward state (about 1e-6 relative), which moves the residuals the
    weight gradient is made of by ~1e-3 px against ~1 px, so entries are held
    to relative 1e-2 above that floor plus 2^-20 of the largest entry (a few
    FP32 roundings of the per-edge products), and the whole gradient to 1e-3
    in norm."""
    need_gpu()
    w = synth.gradient_subwindow(0)
    gp = np.zeros((w.n_frames, 7))
    gd = np.zeros(w.n_patches)
    rng = np.random.default_rng(3)
    gp[w.n_fixed:] = rng.normal(size=(w.n_frames - w.n_fixed, 7))
    gd[:] = rng.normal(size=w.n_patches)
    gy, gwt, st = gpu_vjp(w, gp, gd, precision)
    assert st[0] == 0

    def f(wx):
        p, d = O.solve(wx)
        return float((p * gp).sum() + (d * gd).sum()), float(np.abs(p * gp).sum() + np.abs(d * gd).sum())

    h = 1e-6
    _, mag = f(w)
    floor = _fd_floor(mag, h)
    act = np.nonzero((w.anchor[w.kk] != w.jj) & (w.weights[:, 0] > 0))[0]
    rel = 1e-4 if precision == "fp64" else 1e-2
    ratio, norm_err, bad = {}, {}, []
    for arr, g in (("targets", gy), ("weights", gwt)):
        fl = floor + (2.0 ** -20 * np.abs(g).max() if precision == "fp32" else 0.0)
        r, fds = [], []
        for e in act:
            for c in range(2):
                wp, wm = w.copy(), w.copy()
                getattr(wp, arr)[e, c] += h
                getattr(wm, arr)[e, c] -= h
                fd = (f(wp)[0] - f(wm)[0]) / (2 * h)
                fds.append(fd)
                r.append(abs(fd - g[e, c]) / (rel * abs(fd) + fl))
                if r[-1] >= 1.0:
                    bad.append((arr, int(e), c, fd, float(g[e, c]), fl))
        ratio[arr] = max(r)
        ga = g[act].reshape(-1)
        norm_err[arr] = float(np.linalg.norm(ga - np.asarray(fds)) / np.linalg.norm(fds))
    print(f"{precision} FD check over {len(act)} active edges: worst error / ({rel:g} |fd| + floor): "
          f"targets {ratio['targets']:.3f} weights {ratio['weights']:.3f}; {len(bad)} entries over; "
          f"norm rel err targets {norm_err['targets']:.2e} weights {norm_err['weights']:.2e}")
    assert not bad, bad[:5]
    assert max(norm_err.values()) < (1e-4 if precision == "fp64" else 1e-3)


@pytest.mark.parametrize("shape,precision", [((24, 12, 8), "fp64"), ((40, 16, 16), "fp32"), ((64, 16, 16), "fp32")])
def test_vjp_wide_windows_match_oracle(shape, precision):
    """Windows with more than 21 free frames (n = 132, 228, 372): the reduced
    system gathered into device memory and factorised by panels in both the
    recomputed forward steps and the adjoint steps, the second right-hand side
    solved on the same factor.  Against the oracle's autograd with fixed
    random cotangents: FP64 within 1e-8; FP32 assembly within the change the
    oracle's own product shows when its reduced system is rounded once to
    FP32, times the summation factor sqrt(patches per source frame), and at
    least 1e-4 (as for the loss gradient at 22 x 96)."""
    need_gpu()
    F, ppf, r = shape
    w = synth.make_window(F, ppf, r, seed=[2208, 11, F], outlier_frac=0.1, fp32=True)
    assert 6 * (F - 2) > 126
    rng = np.random.default_rng(F)
    gp = rng.normal(size=(w.n_frames, 7))
    gd = rng.normal(size=w.n_patches)
    gy_ref, gw_ref = O.cotangent_grad(w, gp, gd)
    from paper_2208_04726_amd.solver import Solver, make_batch, capacities_for
    s = Solver(precision=precision, **capacities_for([w]))
    b = make_batch([w], precision)
    gt, gw = s.backward(b, torch.as_tensor(gp), torch.as_tensor(gd))
    torch.cuda.synchronize()
    st = s.status()
    s.close()
    gy, gwt = gt.double().cpu().numpy(), gw.double().cpu().numpy()
    assert st[0] == 0
    if precision == "fp64":
        tol_y = tol_w = 1e-8
    else:
        from tests.rounding import cotangent_grad_rounded, fp32_assembly_factor
        gy32, gw32 = cotangent_grad_rounded(w, gp, gd)
        f = fp32_assembly_factor(w)
        tol_y = max(1e-4, f * rel_err(gy32, gy_ref))
        tol_w = max(1e-4, f * rel_err(gw32, gw_ref))
    eg, ew = rel_err(gy, gy_ref), rel_err(gwt, gw_ref)
    print(f"{F} frames {precision}: vjp rel err targets {eg:.2e} (bound {tol_y:.1e}) weights {ew:.2e} (bound {tol_w:.1e})")
    assert eg < tol_y and ew < tol_w
