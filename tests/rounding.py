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
