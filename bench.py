"""Throughput and latency benchmark of the gfx950 bundle-adjustment solve.

Workload (the headline): batches of method-scale windows, 22 frames x 96
patches per frame, edges to every frame within 13 of the source frame, 10%
outliers, FP32 linearisation and assembly with FP64 reduced-pose Cholesky and
back-substitution, 2 Gauss-Newton iterations; synthetic inputs resident in HBM
before timing.  One step = one solve of the whole batch (every stage of every
iteration of every window).

Also measured in the same run:
  * per-kernel times from HIP events around each launch on its stream, and
    the roofline position of the dominant kernel (the assembly);
  * batched serving: a Poisson trace of windows of uneven size from 64 camera
    streams, served by continuous batching with graph replays, against the
    plain one-window-at-a-time solve on the same trace (p50/p99/p99.9 latency
    from arrival to result on the host), plus closed-loop throughput of both;
  * the FP64 CPU oracle on a bounded sample, on the host cores.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3     # MI355X dense FP32 (matrix cores, and packed vector ALU)
HBM_PEAK_GBS = 8000.0
ASSEMBLY_SOURCES = ("paper_2208_04726_amd/csrc/dpba_assemble.h", "paper_2208_04726_amd/csrc/dpba_common.h",
                    "paper_2208_04726_amd/csrc/dpba_prep.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_assemble_fp32_22x96_b256_hbm_traffic.txt")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def assembly_work(w):
    """Algorithmic work of one assembly launch for window w (one iteration):
    flops = 600 per active edge (linearisation and the per-edge block products)
    + 36 per free frame pair of every patch (the Schur outer products);
    bytes = 24 per edge (kk, jj, target, weight in FP32) + 28 per patch
    (x, y, d as f64 and the anchor) + 56 per frame (pose)."""
    Ea = int((w.anchor[w.kk] != w.jj).sum())
    M, N, nf = w.n_patches, w.n_frames, w.n_fixed
    touched = np.zeros((M, N), bool)
    touched[w.kk, w.jj] = True
    touched[np.arange(M), w.anchor] = True
    f = touched[:, nf:].sum(1).astype(np.float64)
    flops = 600.0 * Ea + 36.0 * float((f * f).sum())
    bytes_ = 24.0 * w.n_edges + 28.0 * M + 56.0 * N
    return flops, bytes_, Ea


def source_digest(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per assembly launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None, "no counter summary"
    kv = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_digest") != source_digest(ASSEMBLY_SOURCES):
        return None, "kernel changed since the counters were taken"
    try:
        return float(kv["bytes_per_launch"]), "rocprofv3 FETCH_SIZE+WRITE_SIZE, copy-calibrated"
    except (KeyError, ValueError):
        return None, "malformed counter summary"


COPY_BYTES = 256 * 2 ** 20


def pmc_workload(args):
    """The program the counter runs profile: a plain device copy of
    COPY_BYTES (calibration of FETCH_SIZE / WRITE_SIZE), then warm-up and
    `--steps` solves of the headline batch."""
    import torch
    from paper_2208_04726_amd import synth
    from paper_2208_04726_amd.solver import Solver, make_batch, capacities_for
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    windows = [synth.method_scale_window(i) for i in range(args.batch)]
    solver = Solver(precision="fp32", iterations=2, schedule=args.schedule, **capacities_for(windows))
    batch = make_batch(windows, "fp32")
    for _ in range(args.warmup + args.steps):
        solver.solve(batch)
    torch.cuda.synchronize()
    log(f"pmc workload done: {args.steps + args.warmup} solves of {args.batch} windows")


def _pmc_rows(path):
    import csv
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            rows.append((r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])))
    return rows


def pmc_summarize(fetch_csv, write_csv, command):
    """Writes the HBM traffic summary of the assembly kernel from the two
    counter runs: per dispatch FETCH_SIZE and WRITE_SIZE (KiB), each scaled by
    what the counter reads for the calibration copy of COPY_BYTES."""
    def per_kernel(rows, counter):
        d = {}
        for name, c, v in rows:
            if c == counter:
                d.setdefault(name, []).append(v)
        return d
    fr = per_kernel(_pmc_rows(fetch_csv), "FETCH_SIZE")
    wr = per_kernel(_pmc_rows(write_csv), "WRITE_SIZE")
    copy = max((k for k in fr if not k.startswith("void dpba::") and "k_" not in k.split("(")[0]),
               key=lambda k: max(fr[k]))
    f_factor = max(fr[copy]) * 1024.0 / COPY_BYTES
    w_factor = max(wr[copy]) * 1024.0 / COPY_BYTES
    asm = [k for k in fr if "k_assemble" in k]
    if not asm:
        raise SystemExit("no k_assemble dispatches in the counter output")
    fetch = float(np.mean(fr[asm[0]])) * 1024.0 / f_factor
    write = float(np.mean(wr[asm[0]])) * 1024.0 / w_factor
    lines = ["# HBM traffic of the assembly kernel (k_assemble), FP32, 256 windows of 22x96, r=13",
             f"# counters: rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE, in separate runs of: {command}",
             f"# calibration: {copy.split('(')[0][:80]} copying {COPY_BYTES} B read FETCH_SIZE "
             f"{max(fr[copy]):.0f} KiB, WRITE_SIZE {max(wr[copy]):.0f} KiB",
             f"kernel = {asm[0].split('(')[0]}",
             f"dispatches = {len(fr[asm[0]])}",
             f"fetch_kib_raw = {np.mean(fr[asm[0]]):.1f}",
             f"write_kib_raw = {np.mean(wr[asm[0]]):.1f}",
             f"fetch_factor = {f_factor:.4f}",
             f"write_factor = {w_factor:.4f}",
             f"fetch_bytes_per_launch = {fetch:.0f}",
             f"write_bytes_per_launch = {write:.0f}",
             f"bytes_per_launch = {fetch + write:.0f}",
             f"source_digest = {source_digest(ASSEMBLY_SOURCES)}"]
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cpu_oracle_baseline(windows, budget_s):
    """The FP64 oracle as it stands, one window after another on the host,
    for about `budget_s` seconds."""
    import torch
    from oracle import ba_oracle as O
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and n < len(windows):
        O.solve(windows[n])
        n += 1
    dt = time.perf_counter() - t0
    return dict(value=round(n / dt, 3), unit="windows/s", cores=int(torch.get_num_threads()), kind="oracle",
                sample=f"first {n} windows of the batch (22x96, r=13), FP64 dense normal equations "
                       f"over all unknowns, 2 iterations each, {dt:.1f} s")


def run_large(args, torch):
    """Eight 64-frame x 256-patch windows (radius 16, 10% outliers), 4
    iterations, one batched solve per step."""
    from paper_2208_04726_amd import synth
    from paper_2208_04726_amd.solver import Solver, make_batch, capacities_for
    t0 = time.perf_counter()
    wins = [synth.large_window(i) for i in range(args.large_windows)]
    log(f"generated {len(wins)} large windows in {time.perf_counter() - t0:.1f}s")
    iters = 4
    solver = Solver(precision="fp32", iterations=iters, schedule="split", **capacities_for(wins))
    batch = make_batch(wins, "fp32")
    stream = torch.cuda.current_stream()
    for _ in range(2):
        solver.solve(batch, stream=stream)
    torch.cuda.synchronize()
    bad = int((solver.status() != 0).sum())
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.large_steps):
        solver.solve(batch, stream=stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / args.large_steps
    # per-kernel breakdown outside the timed loop
    solver.set_timing(True)
    solver.kernel_times()
    for _ in range(args.large_steps):
        solver.solve(batch, stream=stream)
    kt = solver.kernel_times()
    solver.set_timing(False)
    Ea = sum(int((w.anchor[w.kk] != w.jj).sum()) for w in wins)
    fl = by = 0.0
    for w in wins:
        f_, b_, _ = assembly_work(w)
        fl += f_
        by += b_
    asm_ms = kt["assemble"][0] / max(kt["assemble"][1], 1)
    solver.close()
    return {"workload": f"{len(wins)} windows of 64 frames x 256 patches/frame, radius 16, 10% outliers, "
                        "4 GN iterations, FP32 assembly + FP64 372x372 Cholesky",
            "ms_per_solve_batch": round(ms, 4), "windows_per_s": round(len(wins) / (ms / 1e3), 2),
            "edges_per_s": round(Ea * iters / (ms / 1e3), 1), "active_edges_per_window": Ea // len(wins),
            "active_residual_rows_per_window": 2 * Ea // len(wins),
            "kernels": {k: {"ms_per_launch": round(v[0] / v[1], 4), "launches_per_step": v[1] / args.large_steps}
                        for k, v in kt.items() if v[1] > 0},
            "assembly_tflops": round(fl / (asm_ms / 1e3) / 1e12, 3),
            "assembly_algorithmic_hbm_gbs": round(by / (asm_ms / 1e3) / 1e9, 1),
            "status_failures": bad}


def run_serving(args, torch):
    from paper_2208_04726_amd import serve, synth
    t0 = time.perf_counter()
    pool = [serve.request_from_window(synth.serving_window(i), rid=i) for i in range(args.serve_pool)]
    log(f"serving pool of {len(pool)} windows in {time.perf_counter() - t0:.1f}s")
    cap = serve.Capacity(windows=args.serve_slot_windows, frames=args.serve_slot_windows * 22,
                         patches=args.serve_slot_windows * 22 * 96,
                         edges=args.serve_slot_windows * 22 * 96 * 27, frames_per_window=22)
    n = args.serve_warmup + args.serve_requests
    trace = serve.poisson_trace(pool, n, rate=args.serve_rate, n_streams=64, seed=2208)
    closed = serve.poisson_trace(pool, args.serve_closed, rate=float("inf"), n_streams=64, seed=2209)
    out = {"rate_per_s": args.serve_rate, "requests": args.serve_requests, "warmup_requests": args.serve_warmup,
           "streams": 64, "pool_windows": len(pool),
           "mean_edges": round(float(np.mean([p.kk.shape[0] for p in pool])), 1)}

    srv = serve.BatchedServer(cap, n_slots=args.serve_slots, schedule=args.serve_schedule,
                              chunk_frames=args.serve_chunk, use_graph=True)
    srv.run(closed[:64])  # warm the slots and graphs
    srv.batch_sizes.clear()
    t = time.perf_counter()
    res = srv.run(trace)
    wall = time.perf_counter() - t
    bad = sum(1 for r in res.values() if r.status != 0)
    b = serve.latency_summary(res, skip=args.serve_warmup)
    b.update(solves_per_s=round(n / wall, 1), mean_batch=round(float(np.mean(srv.batch_sizes)), 2),
             status_failures=bad)
    t = time.perf_counter()
    srv.batch_sizes.clear()
    srv.run(closed)
    b["closed_loop_solves_per_s"] = round(len(closed) / (time.perf_counter() - t), 1)
    b["closed_loop_mean_batch"] = round(float(np.mean(srv.batch_sizes)), 2)
    b["slot_footprint_mb"] = round(srv.footprint_bytes / 2 ** 20, 1)
    out["batched"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in b.items()}
    out["batched"].update(schedule=args.serve_schedule, slots=args.serve_slots, graph=True)
    log(f"batched serving: {out['batched']}")

    plain = serve.PlainServer(serve.Capacity(1, 22, 22 * 96, 22 * 96 * 27, 22))
    plain.run(closed[:32])
    t = time.perf_counter()
    res = plain.run(trace)
    wall = time.perf_counter() - t
    p = serve.latency_summary(res, skip=args.serve_warmup)
    p.update(solves_per_s=round(n / wall, 1), status_failures=sum(1 for r in res.values() if r.status != 0))
    t = time.perf_counter()
    plain.run(closed)
    p["closed_loop_solves_per_s"] = round(len(closed) / (time.perf_counter() - t), 1)
    out["plain"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in p.items()}
    log(f"plain serving: {out['plain']}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=256, help="windows per step")
    ap.add_argument("--schedule", default="split", choices=["auto", "fused", "split"])
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--serve-warmup", type=int, default=1000)
    ap.add_argument("--serve-closed", type=int, default=2000)
    ap.add_argument("--serve-pool", type=int, default=64)
    ap.add_argument("--serve-slots", type=int, default=2)
    ap.add_argument("--serve-slot-windows", type=int, default=32)
    ap.add_argument("--serve-schedule", default="split", choices=["fused", "split"])
    ap.add_argument("--serve-chunk", type=int, default=4)
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--large-only", action="store_true",
                    help="run only the 64x256 large-window batch (for its profile) and print its record")
    ap.add_argument("--large-windows", type=int, default=8)
    ap.add_argument("--large-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--pmc-workload", action="store_true",
                    help="run only the calibration copy and the solves (for counter runs)")
    ap.add_argument("--pmc-summarize", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--pmc-command", default="python3 bench.py --pmc-workload --steps 3 --warmup 1")
    args = ap.parse_args()
    if args.pmc_summarize:
        pmc_summarize(args.pmc_summarize[0], args.pmc_summarize[1], args.pmc_command)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (windows are independent, "
              "so batches shard across GPUs without communication, but this build measures one GPU)",
              file=sys.stderr)
        sys.exit(2)

    if args.large_only:
        import torch
        print(json.dumps(run_large(args, torch)), flush=True)
        return
    if args.pmc_workload:
        pmc_workload(args)
        return

    import torch
    from paper_2208_04726_amd import synth
    from paper_2208_04726_amd.solver import Solver, make_batch, capacities_for

    iters = 2
    t0 = time.perf_counter()
    windows = [synth.method_scale_window(i) for i in range(args.batch)]
    log(f"generated {len(windows)} windows in {time.perf_counter() - t0:.1f}s")

    solver = Solver(precision="fp32", iterations=iters, schedule=args.schedule, **capacities_for(windows))
    batch = make_batch(windows, "fp32")
    F, P, E = batch.totals
    poses_out = torch.empty((F, 7), dtype=torch.float64, device="cuda")
    depth_out = torch.empty((P,), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        solver.solve(batch, poses_out, depth_out, stream=stream)
    torch.cuda.synchronize()
    n_bad = int((solver.status() != 0).sum())

    # timed region: K steps; the dominant kernel (the assembly) bracketed by
    # events on its launch stream
    solver.set_timing(True, stages=("assemble",))
    solver.kernel_times()
    step_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for a, b in step_ev:
        a.record(stream)
        solver.solve(batch, poses_out, depth_out, stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    kt = solver.kernel_times()
    # per-kernel breakdown: every kernel bracketed, outside the timed region
    solver.set_timing(True)
    n_bd = max(2, args.steps // 2)
    for _ in range(n_bd):
        solver.solve(batch, poses_out, depth_out, stream=stream)
    kt_all = solver.kernel_times()
    solver.set_timing(False)
    per_step = np.array([a.elapsed_time(b) for a, b in step_ev])
    ms_per_step = wall * 1e3 / args.steps
    value = args.batch / (ms_per_step / 1e3)
    log(f"{args.steps} steps: {ms_per_step:.3f} ms/step (events {per_step.mean():.3f}), {value:.0f} windows/s")

    fl = by = 0.0
    Ea_total = 0
    for w in windows:
        f_, b_, ea = assembly_work(w)
        fl += f_
        by += b_
        Ea_total += ea
    asm_ms, asm_n = kt["assemble"]
    launch_ms = asm_ms / max(asm_n, 1)
    achieved = fl / (launch_ms / 1e3) / 1e12
    traffic, traffic_note = measured_traffic()
    kernels = {k: {"ms_per_launch": round(v[0] / v[1], 4), "launches_per_step": v[1] / n_bd}
               for k, v in kt_all.items() if v[1] > 0}

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
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "method-scale BA windows: 22 frames x 96 patches/frame, edge radius 13, "
                               "10% outliers, 2 GN iterations, FP32 assembly + FP64 Cholesky/back-substitution",
                   "windows_per_step": args.batch, "edges_per_window": int(E // args.batch),
                   "schedule": args.schedule},
        "edges_per_s": round(Ea_total * iters / (ms_per_step / 1e3), 1),
        "kernels": kernels,
        "roofline": {"bound": "mfma", "kernel": "k_assemble", "achieved": round(achieved, 3),
                     "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 5),
                     "traffic": traffic, "traffic_note": traffic_note,
                     "flops_per_launch": fl, "algorithmic_bytes_per_launch": by,
                     "launch_ms": round(launch_ms, 4),
                     "algorithmic_hbm_gbs": round(by / (launch_ms / 1e3) / 1e9, 1)},
        "status_failures": n_bad,
    }
    if traffic:
        out["roofline"]["achieved_hbm_gbs"] = round(traffic / (launch_ms / 1e3) / 1e9, 1)
        out["roofline"]["hbm_frac"] = round(traffic / (launch_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 5)
    solver.close()
    del batch, poses_out, depth_out
    torch.cuda.empty_cache()

    if not args.no_large:
        out["large_window"] = run_large(args, torch)
        log(f"large windows: {out['large_window']}")
    if not args.no_serve:
        s = run_serving(args, torch)
        out["serving"] = s
        out["latency_ms"] = {"batched_p50": s["batched"].get("p50_ms"), "batched_p99": s["batched"].get("p99_ms"),
                             "plain_p50": s["plain"].get("p50_ms"), "plain_p99": s["plain"].get("p99_ms")}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_oracle_baseline(windows, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
