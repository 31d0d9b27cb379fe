"""Windows with more than 21 free frames: the reduced system is gathered in
device memory and factorised by the blocked FP64 Cholesky.  Parity with the
dense oracle where it fits, with the block-eliminated oracle at 64 x 256."""
import numpy as np
import pytest
import torch

from oracle import ba_oracle as O
from paper_2208_04726_amd import synth
from tests.gpu_util import compare, need_gpu, solve_gpu
from tests.rounding import check_depths, depth_sensitivity, fp32_assembly_factor, solve_schur_rounded

pytestmark = pytest.mark.gpu

FP64_TOL = (1e-6, 1e-4, 1e-6)
FP32_TOL = (1e-4, 1e-2, 1e-3)


def fp32_tolerance(w, iterations=2):
    """Pose tolerance of FP32 assembly for window w: the fixed FP32 bounds, or
    the change the FP64 oracle itself shows when its reduced system is rounded
    once to FP32 per iteration, times the probabilistic summation factor
    sqrt(patches per source frame) (`fp32_assembly_factor`), whichever is
    larger.  Long windows with few patches per frame have reduced systems with
    condition numbers near 1e7 (scale drift along the trajectory), where one
    FP32 rounding of S alone moves the poses by more than 1e-4 m."""
    pr, dr = O.solve_schur(w, iterations=iterations)
    p32, d32 = solve_schur_rounded(w, iterations=iterations)
    dc, drot, _ = compare(p32, d32, pr, dr)
    f = fp32_assembly_factor(w)
    return max(FP32_TOL[0], f * dc), max(FP32_TOL[1], f * drot)


def _wide(n_frames, ppf, r, seed, fp32=True, n_fixed=2):
    return synth.make_window(n_frames, ppf, r, seed=[2208, 9, seed], outlier_frac=0.1, fp32=fp32,
                             n_fixed=n_fixed)


@pytest.mark.parametrize("chunk_frames", [0, 64])
def test_reduced_system_372_matches_oracle(chunk_frames):
    """S and s of a 64-frame window (n = 372).  With the automatic chunking
    each chunk spans about 34 free frames (one pass of 12 accumulator tiles
    per wave); with one chunk of all 64 frames the FP32 assembly takes four
    tile passes, each keeping its FP64 running sums in the partial block."""
    need_gpu()
    from paper_2208_04726_amd.solver import Solver, make_batch, capacities_for
    w = _wide(64, 16, 16, 0)
    s = Solver(precision="fp32", chunk_frames=chunk_frames, **capacities_for([w]))
    S, sv = s.reduced_system(make_batch([w], "fp32"))
    torch.cuda.synchronize()
    S_ref, s_ref = O.reduced_system(w)
    S, sv = S.cpu().numpy(), sv.cpu().numpy()
    assert S.shape == (372, 372)
    rel_S = np.abs(S - S_ref).max() / np.abs(S_ref).max()
    rel_s = np.abs(sv - s_ref).max() / np.abs(s_ref).max()
    print(f"S rel {rel_S:.2e} s rel {rel_s:.2e}")
    # 16 patches per source frame: n <= 48 FP32 roundings, gamma_n = 2.9e-6 (see test_gpu_parity)
    assert rel_S < 1e-5 and rel_s < 1e-5


def test_372_solve_is_the_solution_of_its_system():
    """One iteration at n = 372: the pose step is the FP64 solution of the
    reduced system the GPU assembled (isolates the blocked Cholesky and the
    triangular solves from FP32 assembly rounding)."""
    need_gpu()
    from paper_2208_04726_amd.solver import Solver, make_batch, capacities_for
    w = _wide(64, 16, 16, 0)
    b = make_batch([w], "fp32")
    s = Solver(precision="fp32", iterations=1, **capacities_for([w]))
    S, sv = s.reduced_system(b)
    po, _ = s.solve(b)
    torch.cuda.synchronize()
    assert (s.status() == 0).all()
    x = -np.linalg.solve(S.cpu().numpy(), sv.cpu().numpy())
    ref = O.retract(torch.as_tensor(w.poses[2:]), torch.as_tensor(x.reshape(-1, 6))).numpy()
    dc, drot = synth.pose_errors(po.cpu().numpy()[2:], ref)
    print(f"step vs solve of own system: {dc:.2e} m {drot:.2e} deg")
    assert dc < 1e-8 and drot < 1e-6


# reduced sizes n = 372, 168, 132, 192, 144: the factorisation's last
# 32-column panel holds two sub-blocks (the second partial), one partial
# sub-block, a short one, a whole panel, and exactly one full sub-block
@pytest.mark.parametrize("shape", [(64, 16, 16), (30, 24, 16), (24, 40, 13), (34, 16, 16), (26, 24, 13)])
def test_fp32_wide_window_matches_oracle(shape):
    need_gpu()
    N, ppf, r = shape
    w = _wide(N, ppf, r, 1)
    out, st = solve_gpu([w], "fp32", "auto")
    assert (st == 0).all()
    pr, dr = O.solve(w)
    dc, drot, dd = compare(out[0][0], out[0][1], pr, dr)
    tol = fp32_tolerance(w)
    print(f"{shape}: {dc:.2e} m {drot:.2e} deg depth {dd:.2e} (tolerance {tol[0]:.1e} m {tol[1]:.1e} deg)")
    assert dc < tol[0] and drot < tol[1]
    check_depths(out[0][1], dr, depth_sensitivity(w), label=str(shape))


def test_fp64_24_frames_matches_oracle():
    """n = 132 in FP64: the blocked Cholesky at FP64 parity."""
    need_gpu()
    w = _wide(24, 12, 8, 2, fp32=False)
    for sched in ("split", "auto"):
        out, st = solve_gpu([w], "fp64", sched)
        assert (st == 0).all()
        pr, dr = O.solve(w)
        dc, drot, dd = compare(out[0][0], out[0][1], pr, dr)
        print(f"fp64 {sched}: {dc:.2e} m {drot:.2e} deg depth {dd:.2e}")
        assert dc < FP64_TOL[0] and drot < FP64_TOL[1] and dd < FP64_TOL[2]


def test_mixed_small_and_wide_windows_alone_equals_batch():
    need_gpu()
    wins = [synth.method_scale_window(3), _wide(40, 16, 16, 3), synth.serving_window(5), _wide(64, 8, 16, 4)]
    batch, st = solve_gpu(wins, "fp32", "split", chunk_frames=2, max_frames_per_window=64)
    assert (st == 0).all()
    for i, w in enumerate(wins):
        alone, st1 = solve_gpu([w], "fp32", "split", chunk_frames=2, max_frames_per_window=64)
        assert (st1 == 0).all()
        assert np.array_equal(alone[0][0], batch[i][0]) and np.array_equal(alone[0][1], batch[i][1]), i


def test_fused_schedule_rejects_wide_windows():
    need_gpu()
    from paper_2208_04726_amd import native
    with pytest.raises(native.BAError) as e:
        solve_gpu([_wide(30, 8, 16, 5)], "fp32", "fused")
    assert e.value.code == native.BA_E_CAPACITY


def test_large_windows_64x256_k4_batch_of_8():
    """Eight 64-frame x 256-patch windows (radius 16, 4 iterations) in one call;
    two of them checked against the block-eliminated FP64 oracle."""
    need_gpu()
    wins = [synth.large_window(i) for i in range(8)]
    out, st = solve_gpu(wins, "fp32", "auto", iterations=4)
    assert (st == 0).all(), st
    for i in range(8):
        pr, dr = O.solve_schur(wins[i], iterations=4)
        dc, drot, dd = compare(out[i][0], out[i][1], pr, dr)
        print(f"large window {i}: {dc:.2e} m {drot:.2e} deg depth {dd:.2e}")
        # the 64 x 256 windows meet the fixed FP32 pose bounds
        assert dc < FP32_TOL[0] and drot < FP32_TOL[1]
        check_depths(out[i][1], dr, depth_sensitivity(wins[i], iterations=4), label=f"large window {i}")
