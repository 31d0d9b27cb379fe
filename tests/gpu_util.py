"""Helpers shared by the GPU tests (no oracle arithmetic here)."""
import numpy as np
import pytest
import torch

from paper_2208_04726_amd import synth


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def solve_gpu(windows, precision="fp32", schedule="auto", iterations=2, **kw):
    from paper_2208_04726_amd.solver import Solver, make_batch, capacities_for
    caps = capacities_for(windows)
    caps.update(kw)
    s = Solver(precision=precision, schedule=schedule, iterations=iterations, **caps)
    b = make_batch(windows, precision)
    po, do = s.solve(b)
    torch.cuda.synchronize()
    st = s.status()
    out = []
    for i, w in enumerate(windows):
        f0, f1 = b.frame_off[i], b.frame_off[i + 1]
        p0, p1 = b.patch_off[i], b.patch_off[i + 1]
        out.append((po[f0:f1].cpu().numpy(), do[p0:p1].cpu().numpy()))
    s.close()
    return out, st


def compare(poses_a, depth_a, poses_b, depth_b):
    dc, dr = synth.pose_errors(poses_a, poses_b)
    dd = float(np.max(np.abs(depth_a - depth_b) / np.maximum(np.abs(depth_b), 1e-12))) if len(depth_b) else 0.0
    return dc, dr, dd
