"""Throughput benchmark of the gfx950 bundle-adjustment solve.

Workload: batches of method-scale windows (22 frames x 96 patches per frame,
edges to every frame within 13 of the source frame, 10% outliers, FP32
assembly with FP64 reduced-pose Cholesky, 2 Gauss-Newton iterations), all
inputs synthetic and resident in HBM before timing.  One step = one solve of
the whole batch (every stage of every iteration for every window).

Prints one JSON line.  Also reports the roofline position of the solve
kernel, per-window latency of batched vs one-window-at-a-time solves, and
the FP64 CPU oracle timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_MFMA_PEAK_TFLOPS = 157.3     # MI355X dense FP32 matrix peak
HBM_PEAK_GBS = 8000.0


def algorithmic_work(windows, iterations):
    """Algorithmic flops and HBM bytes of one solve of `windows`.

    flops per iteration and window:
      * 230 per active edge (reprojection 30, Jacobian rows 40, J_d^T W J_d and
        J_d^T W r 8, E_j 12, E_i = -Ad^T E_j 36, J_j^T W J_j 84, J_j^T W r 24);
      * sum over patches of (6 f_k + 1)^2, the lower-triangle multiply-adds of
        the patch's depth-eliminated outer product (f_k = free frames it touches);
      * n^3 / 3 for the Cholesky of the reduced pose system (n = 6 free frames);
      * 60 per active edge of the depth back-substitution.
    bytes: every input read once per iteration (kk, jj, targets, weights:
    24 B per edge in FP32; patches 24 B + anchor 4 B per patch; poses 56 B per
    frame) and the outputs written once (56 B per frame, 8 B per patch)."""
    fl = 0.0
    by = 0.0
    for w in windows:
        ii = w.anchor[w.kk]
        act = (ii != w.jj) & (w.weights[:, 0] > 0)
        Ea = float(act.sum())
        nf = w.n_fixed
        sq = 0.0
        for k in range(w.n_patches):
            fr = set(w.jj[w.kk == k].tolist()) | {int(w.anchor[k])}
            f = sum(1 for a in fr if a >= nf)
            sq += (6 * f + 1) ** 2
        n = 6 * (w.n_frames - nf)
        fl += iterations * (230 * Ea + sq + n ** 3 / 3 + 60 * Ea)
        by += iterations * (24 * w.n_edges + 28 * w.n_patches + 56 * w.n_frames) + 56 * w.n_frames + 8 * w.n_patches
    return fl, by


def patch_sq_fast(w):
    """sum_k (6 f_k + 1)^2 without a Python loop over patches."""
    nf = w.n_fixed
    M = w.n_patches
    touched = np.zeros((M, w.n_frames), bool)
    touched[w.kk, w.jj] = True
    touched[np.arange(M), w.anchor] = True
    f = touched[:, nf:].sum(1)
    return float(((6 * f + 1) ** 2).sum())


def work_fast(windows, iterations):
    fl = by = 0.0
    for w in windows:
        act = (w.anchor[w.kk] != w.jj) & (w.weights[:, 0] > 0)
        Ea = float(act.sum())
        n = 6 * (w.n_frames - w.n_fixed)
        fl += iterations * (290 * Ea + patch_sq_fast(w) + n ** 3 / 3)
        by += iterations * (24 * w.n_edges + 28 * w.n_patches + 56 * w.n_frames) + 56 * w.n_frames + 8 * w.n_patches
    return fl, by


def cpu_oracle_baseline(windows, budget_s=15.0):
    """The FP64 oracle on the host, one window after another, for about
    `budget_s` seconds."""
    import torch
    from oracle import ba_oracle as O
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and n < len(windows):
        O.solve(windows[n])
        n += 1
    dt = time.perf_counter() - t0
    return dict(value=n / dt, unit="windows/s", cores=int(torch.get_num_threads()), kind="oracle",
                sample=f"{n} method-scale windows (22x96, r=13), FP64 dense normal equations, "
                       f"{dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=256, help="windows per step")
    ap.add_argument("--schedule", default="fused", choices=["auto", "fused", "split"])
    ap.add_argument("--latency-samples", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2208_04726_amd import synth
    from paper_2208_04726_amd.solver import Solver, make_batch, capacities_for

    iters = 2
    t0 = time.perf_counter()
    windows = [synth.method_scale_window(i) for i in range(args.batch)]
    gen_s = time.perf_counter() - t0
    print(f"[bench] generated {len(windows)} windows in {gen_s:.1f}s", file=sys.stderr, flush=True)

    caps = capacities_for(windows)
    solver = Solver(precision="fp32", iterations=iters, schedule=args.schedule, **caps)
    batch = make_batch(windows, "fp32")
    F, P, E = batch.totals
    poses_out = torch.empty((F, 7), dtype=torch.float64, device="cuda")
    depth_out = torch.empty((P,), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        solver.solve(batch, poses_out, depth_out)
    torch.cuda.synchronize()
    st = solver.status()
    n_bad = int((st != 0).sum())

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    step_ms = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        e_a = torch.cuda.Event(enable_timing=True)
        e_b = torch.cuda.Event(enable_timing=True)
        e_a.record(stream)
        solver.solve(batch, poses_out, depth_out)
        e_b.record(stream)
        step_ms.append((e_a, e_b))
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    total_ms = ev0.elapsed_time(ev1)
    per_step = [a.elapsed_time(b) for a, b in step_ms]
    ms_per_step = total_ms / args.steps
    value = args.batch / (ms_per_step / 1e3)

    flops, bytes_ = work_fast(windows, iters)
    kern_ms = float(np.mean(per_step))
    achieved_tflops = flops / (kern_ms / 1e3) / 1e12
    E_active = sum(int(((w.anchor[w.kk] != w.jj)).sum()) for w in windows)

    # latency: one window per call on the plain (split) schedule vs the batched step
    plain = Solver(precision="fp32", iterations=iters, schedule="split", **capacities_for(windows[:1]))
    one = make_batch(windows[:1], "fp32")
    lat = []
    for i in range(10):
        plain.solve(one)
    torch.cuda.synchronize()
    for i in range(args.latency_samples):
        t1 = time.perf_counter()
        plain.solve(one)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
    lat = np.asarray(lat)
    batched_lat = np.asarray(per_step)

    out = {
        "metric": "BA window solves/s (22f x 96p, 2 GN iters); p99 latency batched vs plain",
        "value": round(value, 1),
        "unit": "windows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32-assembly/fp64-cholesky",
        "data": "synthetic",
        "config": {"workload": "method-scale BA windows: 22 frames x 96 patches/frame, radius 13, "
                               "10% outliers, 2 GN iterations, FP32 assembly + FP64 Cholesky",
                   "windows_per_step": args.batch, "edges_per_window": int(E // args.batch),
                   "schedule": args.schedule},
        "edges_per_s": round(E_active * iters / (ms_per_step / 1e3), 1),
        "latency_ms": {
            "batched_step_p50": round(float(np.percentile(batched_lat, 50)), 4),
            "batched_step_p99": round(float(np.percentile(batched_lat, 99)), 4),
            "plain_window_p50": round(float(np.percentile(lat, 50)), 4),
            "plain_window_p99": round(float(np.percentile(lat, 99)), 4),
        },
        "roofline": {"bound": "mfma", "achieved": round(achieved_tflops, 3),
                     "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved_tflops / FP32_MFMA_PEAK_TFLOPS, 5), "traffic": None,
                     "hbm_gbs_algorithmic": round(bytes_ / (kern_ms / 1e3) / 1e9, 2)},
        "status_failures": n_bad,
        "wall_s": round(wall, 3),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_oracle_baseline(windows, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
