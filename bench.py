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
  * parity of reported results against the FP64 oracle (pose m / deg and
    relative inverse depth, per record);
  * the plain FP64 8x16 windows, the adjoint (ba_backward) per window, the
    correlation features (Eq. 4) and the soft aggregation (Eq. 5) of the
    method-scale patch graph;
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


LARGE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_assemble_fp32_64x256_b8_hbm_traffic.txt")
MIX_FILE = os.path.join(ROOT, "profiles", "k_assemble_fp32_22x96_b256_instruction_mix.txt")


def _summary(path):
    """key = value lines of a committed counter summary, or None when it is
    missing or was taken on other assembly sources than the current ones."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.split("(")[0].strip()
    return kv if kv.get("source_digest") == source_digest(ASSEMBLY_SOURCES) else None


def measured_traffic(path=TRAFFIC_FILE):
    """HBM bytes per assembly launch from a committed rocprofv3 counter
    summary, if it was taken on the current kernel sources; else None."""
    if not os.path.exists(path):
        return None, "no counter summary"
    kv = _summary(path)
    if kv is None:
        return None, "kernel changed since the counters were taken"
    try:
        return float(kv["bytes_per_launch"]), "rocprofv3 FETCH_SIZE+WRITE_SIZE, copy-calibrated"
    except (KeyError, ValueError):
        return None, "malformed counter summary"


def assembly_bound():
    """The unit the assembly is priced against, from the committed
    instruction-mix counters of the current sources."""
    kv = _summary(MIX_FILE)
    if kv is None:
        return "alu", "no instruction-mix counters of the current sources"
    return "alu", (f"rocprofv3 SQ counters: {float(kv['valu_to_mfma_insts']):.1f} VALU per MFMA instruction, "
                   f"VALU issue {float(kv['valu_issue_fraction']):.3f} and MFMA busy "
                   f"{float(kv['mfma_busy_fraction']):.3f} of the cycles per SIMD: VALU-dominated and "
                   f"latency-bound, priced against the FP32 arithmetic peak")


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
    if args.pmc_target == "agg":
        for _ in range(args.warmup + args.steps):
            run_aggregation_launch(torch, 0)
            run_aggregation_launch(torch, 1)
            run_aggregation_launch(torch, 0, graph_ready=True)
            run_aggregation_launch(torch, 1, graph_ready=True)
        torch.cuda.synchronize()
        log(f"pmc workload done: {args.steps + args.warmup} aggregation calls per mode")
        return
    if args.pmc_target == "corr":
        for _ in range(args.warmup + args.steps):
            run_correlation_launch(torch)
        torch.cuda.synchronize()
        log(f"pmc workload done: {args.steps + args.warmup} correlation launches")
        return
    if args.pmc_target == "large":
        windows = [synth.large_window(i) for i in range(args.large_windows)]
        iters = 4
    else:
        windows = [synth.method_scale_window(i) for i in range(args.batch)]
        iters = 2
    solver = Solver(precision="fp32", iterations=iters, schedule=args.schedule, **capacities_for(windows))
    batch = make_batch(windows, "fp32")
    for _ in range(args.warmup + args.steps):
        solver.solve(batch)
    torch.cuda.synchronize()
    log(f"pmc workload done: {args.steps + args.warmup} solves of {len(windows)} windows")


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


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_job(job):
    """One oracle solve in a worker process (one thread): (kind, id) -> s."""
    import torch
    torch.set_num_threads(1)
    from oracle import ba_oracle as O
    from paper_2208_04726_amd import synth
    kind, i = job
    w = {"cfg1": synth.method_scale_window, "cfg0": synth.plain_fp64_window}[kind](i)
    t = time.perf_counter()
    O.solve(w)
    return time.perf_counter() - t


def cpu_oracle_baseline(budget_s):
    """The FP64 oracle as it stands, on the host cores, before the GPU is
    touched: all-core throughput on 22x96 windows (one window per process,
    one thread each, every core of the affinity mask, for about `budget_s`
    seconds), and one-thread latency per window of the 22x96, 8x16 and
    64x256 windows (the last by the oracle's block-eliminated solve)."""
    import multiprocessing as mp
    import torch
    cores = len(os.sched_getaffinity(0))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    done = 0
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_job, [("cfg0", i) for i in range(cores)])     # start-up outside the clock
        t0 = time.perf_counter()
        it = pool.imap_unordered(_oracle_job, [("cfg1", i) for i in range(100000)])
        for _ in it:
            done += 1
            if time.perf_counter() - t0 >= budget_s:
                break
        dt = time.perf_counter() - t0
        pool.terminate()
    from oracle import ba_oracle as O
    from paper_2208_04726_amd import synth
    nthreads = torch.get_num_threads()
    torch.set_num_threads(1)
    lat = {}
    for name, make, solve, n in (("cfg1_22x96", synth.method_scale_window, lambda w: O.solve(w), 3),
                                 ("cfg0_8x16", synth.plain_fp64_window, lambda w: O.solve(w), 20),
                                 ("cfg4_64x256_k4", synth.large_window,
                                  lambda w: O.solve_schur(w, iterations=4), 1)):
        ws = [make(i) for i in range(n)]
        t = time.perf_counter()
        for w in ws:
            solve(w)
        lat[name] = round((time.perf_counter() - t) * 1e3 / n, 2)
    torch.set_num_threads(nthreads)
    log(f"cpu oracle: {done} windows in {dt:.1f}s on {cores} processes; 1-thread ms/window {lat}")
    return dict(value=round(done / dt, 3), unit="windows/s", cores=cores, kind="oracle",
                sample=f"{done} windows of 22x96 (r=13) in {dt:.1f} s, one window per process, one thread "
                       f"each, on every core of the affinity mask; FP64 dense normal equations over all "
                       f"unknowns, 2 iterations",
                cpu_model=_cpu_model(), single_thread_ms_per_window=lat)


def pose_depth_errors(po, do, pr, dr):
    """Max camera-centre error (m), rotation error (deg) and relative inverse-
    depth error of a solved window against the oracle's."""
    from paper_2208_04726_amd import synth
    dc, drot = synth.pose_errors(po, pr)
    dd = float(np.max(np.abs(do - dr) / np.abs(dr))) if len(dr) else 0.0
    return dc, drot, dd


def parity_record(pairs, label):
    """{worst pose m, deg, depth rel} over (gpu poses, gpu depth, oracle poses,
    oracle depth) tuples."""
    e = np.array([pose_depth_errors(*p) for p in pairs])
    return {"windows": len(pairs), "max_pose_m": float(e[:, 0].max()), "max_rot_deg": float(e[:, 1].max()),
            "max_depth_rel": float(e[:, 2].max()), "reference": label}


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
    large_traffic, _ = measured_traffic(LARGE_TRAFFIC_FILE)
    po, do = solver.solve(batch, stream=stream)
    torch.cuda.synchronize()
    f1, p1 = int(batch.frame_off[1]), int(batch.patch_off[1])
    out0 = (po[:f1].cpu().numpy(), do[:p1].cpu().numpy())
    solver.close()
    from oracle import ba_oracle as O
    pr, dr = O.solve_schur(wins[0], iterations=iters)
    parity = parity_record([(out0[0], out0[1], pr, dr)], "oracle block-eliminated FP64 solve, window 0")
    return {"workload": f"{len(wins)} windows of 64 frames x 256 patches/frame, radius 16, 10% outliers, "
                        "4 GN iterations, FP32 assembly + FP64 372x372 Cholesky",
            "ms_per_solve_batch": round(ms, 4), "windows_per_s": round(len(wins) / (ms / 1e3), 2),
            "edges_per_s": round(Ea * iters / (ms / 1e3), 1), "active_edges_per_window": Ea // len(wins),
            "active_residual_rows_per_window": 2 * Ea // len(wins),
            "kernels": {k: {"ms_per_launch": round(v[0] / v[1], 4), "launches_per_step": v[1] / args.large_steps}
                        for k, v in kt.items() if v[1] > 0},
            "assembly_tflops": round(fl / (asm_ms / 1e3) / 1e12, 3),
            "assembly_algorithmic_hbm_gbs": round(by / (asm_ms / 1e3) / 1e9, 1),
            "assembly_counter_hbm_gbs": (round(large_traffic / (asm_ms / 1e3) / 1e9, 1) if large_traffic else None),
            "assembly_counter_bytes_per_launch": large_traffic,
            "assembly_algorithmic_bytes_per_launch": by,
            "status_failures": bad, "parity": parity}


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
    out["batched"].update(schedule=args.serve_schedule, slots=len(srv.slots), graph=True)
    log(f"batched serving: {out['batched']}")
    # parity of served results: the first request of four pool windows
    from oracle import ba_oracle as O
    where = {id(p.poses): i for i, p in enumerate(pool)}
    seen, pairs = set(), []
    for r in trace[args.serve_warmup:]:
        pi = where[id(r.poses)]
        if pi in seen:
            continue
        seen.add(pi)
        pr, dr = O.solve(synth.serving_window(pi))
        pairs.append((res[r.rid].poses, res[r.rid].depth, pr, dr))
        if len(pairs) == 4:
            break
    out["parity"] = parity_record(pairs, "oracle dense FP64 solve of four served requests")
    # a rate at which continuous batching engages
    fast = serve.poisson_trace(pool, args.serve_fast_requests, rate=args.serve_fast_rate, n_streams=64, seed=2210)
    srv.batch_sizes.clear()
    t = time.perf_counter()
    res_f = srv.run(fast)
    wall = time.perf_counter() - t
    f = serve.latency_summary(res_f, skip=args.serve_fast_requests // 10)
    f.update(rate_per_s=args.serve_fast_rate, requests=args.serve_fast_requests,
             solves_per_s=round(len(fast) / wall, 1), mean_batch=round(float(np.mean(srv.batch_sizes)), 2),
             status_failures=sum(1 for r in res_f.values() if r.status != 0))
    out["batched_fast"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in f.items()}
    log(f"batched serving at {args.serve_fast_rate:.0f}/s: {out['batched_fast']}")

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


def run_plain_fp64(args, torch):
    """8-frame x 16-patch FP64 windows: batched solves/s, one-window latency,
    and parity of four windows against the dense oracle."""
    from oracle import ba_oracle as O
    from paper_2208_04726_amd import synth
    from paper_2208_04726_amd.solver import Solver, make_batch, capacities_for
    wins = [synth.plain_fp64_window(i) for i in range(args.batch)]
    solver = Solver(precision="fp64", iterations=2, schedule="split", **capacities_for(wins))
    batch = make_batch(wins, "fp64")
    stream = torch.cuda.current_stream()
    for _ in range(3):
        po, do = solver.solve(batch, stream=stream)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        solver.solve(batch, po, do, stream=stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / args.steps
    bad = int((solver.status() != 0).sum())
    pairs = []
    pn, dn = po.cpu().numpy(), do.cpu().numpy()
    for i in range(4):
        f0, f1 = batch.frame_off[i], batch.frame_off[i + 1]
        p0, p1 = batch.patch_off[i], batch.patch_off[i + 1]
        pr, dr = O.solve(wins[i])
        pairs.append((pn[f0:f1], dn[p0:p1], pr, dr))
    solver.close()
    one = Solver(precision="fp64", iterations=2, schedule="split", **capacities_for(wins[:1]))
    b1 = make_batch(wins[:1], "fp64")
    for _ in range(3):
        o1 = one.solve(b1, stream=stream)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(50):
        one.solve(b1, *o1, stream=stream)
        torch.cuda.synchronize()
    ms1 = (time.perf_counter() - t) * 1e3 / 50
    one.close()
    return {"workload": f"{args.batch} windows of 8 frames x 16 patches, radius 3, FP64, 2 GN iterations",
            "ms_per_solve_batch": round(ms, 4), "windows_per_s": round(args.batch / (ms / 1e3), 1),
            "single_window_ms": round(ms1, 4), "status_failures": bad,
            "parity": parity_record(pairs, "oracle dense FP64 solve, windows 0-3")}


def run_backward(args, torch):
    """ba_backward (recomputed iterates, adjoint) of 22x96 windows in FP32 and
    FP64, 32 windows per call, fixed random cotangents; parity of window 0
    against the oracle's vector-Jacobian product."""
    from oracle import ba_oracle as O
    from paper_2208_04726_amd import synth
    from paper_2208_04726_amd.solver import Solver, make_batch, capacities_for
    n = 32
    wins = [synth.method_scale_window(i) for i in range(n)]
    rng = np.random.default_rng(11)
    out = {"workload": f"{n} windows of 22 frames x 96 patches, 2 GN iterations, VJP to targets and weights"}
    w0 = wins[0]
    gp0 = rng.normal(size=(w0.n_frames, 7))
    gd0 = rng.normal(size=w0.n_patches)
    gy_ref, gw_ref = O.cotangent_grad(w0, gp0, gd0)
    for prec in ("fp32", "fp64"):
        solver = Solver(precision=prec, iterations=2, schedule="split", **capacities_for(wins))
        batch = make_batch(wins, prec)
        F, P, _ = batch.totals
        gp = torch.as_tensor(np.concatenate([gp0, rng.normal(size=(F - w0.n_frames, 7))]), device="cuda")
        gd = torch.as_tensor(np.concatenate([gd0, rng.normal(size=P - w0.n_patches)]), device="cuda")
        for _ in range(2):
            gt, gw = solver.backward(batch, gp, gd)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(5):
            gt, gw = solver.backward(batch, gp, gd)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / 5
        E0 = w0.n_edges
        g_t = gt[:E0].double().cpu().numpy()
        g_w = gw[:E0].double().cpu().numpy()
        rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
        out[prec] = {"ms_per_call": round(ms, 4), "ms_per_window": round(ms / n, 5),
                     "vjp_rel_err_targets": rel(g_t, gy_ref), "vjp_rel_err_weights": rel(g_w, gw_ref),
                     "status_failures": int((solver.status() != 0).sum())}
        solver.close()
    return out


_CORR = {}


def run_correlation_launch(torch):
    """One correlation launch (and one pooling launch) on the method-scale
    correlation workload, its device buffers made on first use."""
    from paper_2208_04726_amd import corr, synth
    if not _CORR:
        wl = synth.method_scale_correlation(0)
        dev = lambda a, d: torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=d).contiguous()
        _CORR.update(wl=wl, f0=dev(wl.fmap0, torch.bfloat16), f1=dev(wl.fmap1, torch.bfloat16),
                     g=dev(wl.gmap, torch.bfloat16), c=dev(wl.coords, torch.float32),
                     kk=dev(wl.kk, torch.int32), jj=dev(wl.jj, torch.int32))
        _CORR["out"] = torch.empty((wl.n_edges, 2, 9, 7, 7), dtype=torch.float32, device="cuda")
        _CORR["pooled"] = torch.empty_like(_CORR["f1"])
    d = _CORR
    corr.correlation(d["f0"], d["f1"], d["wl"].scale1, d["g"], d["c"], d["kk"], d["jj"], out=d["out"])
    corr.avg_pool(d["f0"], d["wl"].scale1, out=d["pooled"])


def run_correlation(args, torch):
    """Correlation features (Eq. 4) of the 22 x 96, radius-13 patch graph:
    39,552 edges, 3x3 patches, 128 channels, 160x120 and 40x30 maps in bf16;
    the second level made by the pooling kernel; HIP events around each
    launch; parity of 64 sampled edges against the oracle."""
    from oracle import corr_oracle as C
    from paper_2208_04726_amd import corr, synth
    wl = synth.method_scale_correlation(0)
    dev = lambda a, d: torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=d).contiguous()
    f0 = dev(wl.fmap0, torch.bfloat16)
    f1 = dev(wl.fmap1, torch.bfloat16)
    g = dev(wl.gmap, torch.bfloat16)
    c = dev(wl.coords, torch.float32)
    kk, jj = dev(wl.kk, torch.int32), dev(wl.jj, torch.int32)
    out = torch.empty((wl.n_edges, 2, 9, 7, 7), dtype=torch.float32, device="cuda")
    pooled = torch.empty_like(f1)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        corr.correlation(f0, f1, wl.scale1, g, c, kk, jj, out=out)
        corr.avg_pool(f0, wl.scale1, out=pooled)
    torch.cuda.synchronize()
    reps = 20
    mk = lambda: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    ev, evp = mk(), mk()
    for (a, b), (pa, pb) in zip(ev, evp):
        a.record(stream)
        corr.correlation(f0, f1, wl.scale1, g, c, kk, jj, out=out)
        b.record(stream)
        pa.record(stream)
        corr.avg_pool(f0, wl.scale1, out=pooled)
        pb.record(stream)
    torch.cuda.synchronize()
    avg = lambda evs: float(np.mean([a.elapsed_time(b) for a, b in evs]))
    ms, ms_pool = avg(ev), avg(evp)
    E = wl.n_edges
    nbytes = lambda a: int(np.prod(a.shape))
    by = (2 * nbytes(wl.fmap0) + 2 * nbytes(wl.fmap1) + 2 * nbytes(wl.gmap) + 4 * nbytes(wl.coords)
          + 8 * E + 4 * E * 2 * 9 * 49)
    by_pool = 2 * nbytes(wl.fmap0) + 2 * nbytes(wl.fmap1)
    got = out.cpu().numpy().astype(np.float64)
    sel = np.sort(np.random.default_rng(3).choice(E, 64, replace=False))
    args_ = ([wl.fmap0, wl.fmap1], [1, wl.scale1], wl.gmap, wl.coords[sel], wl.kk[sel], wl.jj[sel])
    ref, mag = C.correlation(*args_), C.correlation_abs(*args_)
    gam = 132 * 2.0 ** -24 / (1 - 132 * 2.0 ** -24)
    gbs = by / (ms / 1e3) / 1e9
    return {"workload": "correlation features, 22 frames x 96 patches, radius 13: 39,552 edges, 3x3 patches, "
                        "D=128, 160x120 and 40x30 bf16 maps, 2 levels x 9 pixels x 7x7 per edge, FP32 out",
            "ms_per_launch": round(ms, 4), "edges_per_s": round(E / (ms / 1e3), 1),
            "algorithmic_bytes_per_launch": by, "achieved_hbm_gbs": round(gbs, 1),
            "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "pool_ms_per_launch": round(ms_pool, 4),
            "pool_hbm_gbs": round(by_pool / (ms_pool / 1e3) / 1e9, 1),
            "parity": {"edges": int(len(sel)), "max_abs_err": float(np.abs(got[sel] - ref).max()),
                       "max_err_over_bound": float((np.abs(got[sel] - ref) / (gam * mag + 1e-300)).max()),
                       "bound": "gamma_(D+4) x summed magnitudes"}}


_AGG = {}


def run_aggregation_launch(torch, mode, graph_ready=False):
    """One soft aggregation of the method-scale workload (buffers made on
    first use)."""
    from paper_2208_04726_amd import agg, synth
    if not _AGG:
        wl = synth.method_scale_aggregation(0)
        dev = lambda a, d: torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=d).contiguous()
        _AGG.update(wl=wl, x=dev(wl.x, torch.bfloat16), kk=dev(wl.kk, torch.int32), jj=dev(wl.jj, torch.int32),
                    anchor=dev(wl.anchor, torch.int32), w=[dev(w, torch.bfloat16) for w in wl.w],
                    b=[dev(b, torch.float32) for b in wl.b])
        _AGG["out"] = torch.empty((wl.n_edges, wl.x.shape[1]), dtype=torch.float32, device="cuda")
        nb = max(agg.workspace_bytes(m, wl.x.shape[1], wl.n_edges, len(wl.anchor), wl.n_frames) for m in (0, 1))
        _AGG["ws"] = [torch.empty((nb,), dtype=torch.uint8, device="cuda") for _ in (0, 1)]
    d = _AGG
    agg.softagg(mode, d["x"], d["kk"], d["jj"], d["anchor"], d["wl"].n_frames, d["w"], d["b"], out=d["out"],
                workspace=d["ws"][mode], graph_ready=graph_ready)


def run_aggregation(args, torch):
    """Soft aggregation (Eq. 5) of the 22 x 96, radius-13 patch graph: 39,552
    edges, 384-channel bf16 hidden states, both neighbourhood kinds; HIP
    events around each call; parity of 256 sampled edges against the
    oracle."""
    from oracle import agg_oracle as A
    out = {"workload": "soft aggregation, 22 frames x 96 patches, radius 13: 39,552 edges, 384-channel bf16 hidden "
                       "states, gate/value/output layers 384x384 bf16, FP32 sums and output"}
    stream = torch.cuda.current_stream()
    for mode, name in ((0, "patch"), (1, "frame")):
        for _ in range(3):
            run_aggregation_launch(torch, mode)
        torch.cuda.synchronize()
        mk = lambda: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
        ev, evr = mk(), mk()
        for (a, b), (ra, rb) in zip(ev, evr):
            a.record(stream)
            run_aggregation_launch(torch, mode)
            b.record(stream)
            ra.record(stream)
            run_aggregation_launch(torch, mode, graph_ready=True)
            rb.record(stream)
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        ms_r = float(np.mean([a.elapsed_time(b) for a, b in evr]))
        wl = _AGG["wl"]
        E, D = wl.x.shape
        key = A.group_keys(mode, wl.kk, wl.jj, wl.anchor, wl.n_frames)
        G = len(np.unique(key))
        flops = 2.0 * E * D * 2 * D + 2.0 * G * D * D
        by = 2.0 * E * D + 4.0 * E * D + 3 * 2.0 * D * D + 8.0 * E
        got = _AGG["out"].cpu().numpy().astype(np.float64)
        ref = A.soft_aggregate(mode, wl.x, wl.kk, wl.jj, wl.anchor, wl.n_frames, wl.w[0], wl.b[0], wl.w[1], wl.b[1],
                               wl.w[2], wl.b[2])
        out[name] = {"ms_per_call": round(ms, 4), "ms_per_call_graph_reused": round(ms_r, 4),
                     "edges_per_s": round(E / (ms / 1e3), 1), "neighbourhoods": G,
                     "matrix_tflops": round(flops / (ms_r / 1e3) / 1e12, 2),
                     "algorithmic_hbm_gbs": round(by / (ms_r / 1e3) / 1e9, 1),
                     "parity_max_abs_err": float(np.abs(got - ref).max()),
                     "parity_max_rel_err": float((np.abs(got - ref) / np.maximum(np.abs(ref), 1e-3)).max())}
    return out


def run_driver(args, torch):
    """The sliding-window driver (Sec. 3.3) stepping `vo_streams` camera
    streams together: 22-keyframe windows of 96 patches, radius 13, two
    Gauss-Newton iterations per frame, flow-based keyframe removal.  Every
    vo_step call waits for its step, so host wall clock per step is the
    latency of one frame for every stream.  Parity: stream 0's final window
    (FP64) against the driver oracle."""
    from oracle import vo_oracle as V
    from paper_2208_04726_amd import synth
    from paper_2208_04726_amd.vo import Driver
    S, warm, timed = args.vo_streams, 25, 30
    T = warm + timed + 1
    out = {"workload": f"{S} camera streams stepped together, 22-keyframe windows x 96 patches, radius 13, "
                       f"2 GN iterations per frame; {T - 1} frames per stream, the first {warm} untimed "
                       "(windows fill), 16 distinct synthetic streams replicated"}
    for prec in ("fp32", "fp64"):
        base = [synth.make_stream(T, 96, seed=[2208, 30, i], fp32=prec == "fp32") for i in range(16)]
        drv = Driver([base[i % 16] for i in range(S)], precision=prec, track_trajectory=False)
        ts = []
        for t in range(warm + timed):
            a = time.perf_counter()
            drv.step(np.full(S, t, np.int32))
            ts.append(time.perf_counter() - a)
        ms = 1e3 * float(np.mean(ts[warm:]))
        n, kf, flow, rem = drv.read()
        rec = {"ms_per_step": round(ms, 4), "frames_per_s": round(S / (ms / 1e3), 1),
               "mean_keyframes": round(float(n.mean()), 2), "status_nonzero": int((drv.status() != 0).sum())}
        if prec == "fp64":
            o = V.StreamOracle(base[0], window=22, radius=13)
            for t in range(warm + timed):
                r = o.step(t)
            k = len(r["kf"])
            poses, depth, eg, ef = drv.window(0)
            dc, dr = synth.pose_errors(poses[:k], r["poses"])
            rec["parity_stream0"] = {
                "keyframes_match": kf[0, :k].tolist() == r["kf"] and int(n[0]) == k,
                "edges_match": sorted(zip(eg.tolist(), ef.tolist())) == r["edges"],
                "max_center_err_m": float(dc), "max_rot_err_deg": float(dr),
                "max_depth_rel_err": float(np.max(np.abs(depth[:k * 96] - r["depth"]) / np.abs(r["depth"])))}
        drv.close()
        out[prec] = rec
        del base
    return out


def run_stream_serving(args, torch):
    """Stateful serving of camera streams (serve.StreamServer): frames arrive
    open-loop at a fixed rate per stream with random phases, every step takes
    the oldest waiting frame of each stream; windows stay on the device.
    Latency = arrival to the end of the step that took the frame, over frames
    25 and later (full windows).  Baseline at 16 streams: one driver per
    stream, one frame per step (serve.PlainStreamServer)."""
    from paper_2208_04726_amd import synth
    from paper_2208_04726_amd.serve import (PlainStreamServer, StreamServer, frame_latency_summary,
                                             frame_trace)
    from paper_2208_04726_amd.vo import Driver
    F = 80
    base = [synth.make_stream(F + 2, 96, seed=[2208, 30, i], fp32=True) for i in range(16)]
    out = {"workload": f"camera streams of 22-keyframe windows x 96 patches, radius 13, FP32 assembly; {F} frames "
                       "per stream at a fixed rate with random phases and 10% jitter; latency over frames 25+"}
    for S, fps in ((256, 60.0), (256, 120.0), (16, 60.0)):
        drv = Driver([base[i % 16] for i in range(S)], precision="fp32", track_trajectory=False)
        reqs = frame_trace(S, F, fps, seed=S)
        t = time.perf_counter()
        res = StreamServer(drv).run(reqs)
        wall = time.perf_counter() - t
        rec = frame_latency_summary(res, min_frame=25)
        rec.update(offered_frames_per_s=S * fps, served_frames_per_s=round(len(reqs) / wall, 1))
        out[f"batched_{S}x{int(fps)}fps"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in rec.items()}
        drv.close()
        if S == 16:
            drivers = [Driver([base[i]], precision="fp32", track_trajectory=False) for i in range(S)]
            t = time.perf_counter()
            res = PlainStreamServer(drivers).run(reqs)
            wall = time.perf_counter() - t
            rec = frame_latency_summary(res, min_frame=25)
            rec.update(offered_frames_per_s=S * fps, served_frames_per_s=round(len(reqs) / wall, 1))
            out[f"plain_{S}x{int(fps)}fps"] = {k: (round(v, 4) if isinstance(v, float) else v)
                                               for k, v in rec.items()}
            for d in drivers:
                d.close()
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
    ap.add_argument("--serve-fast-rate", type=float, default=20000.0)
    ap.add_argument("--serve-fast-requests", type=int, default=20000)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the plain FP64, backward, correlation, aggregation and driver records")
    ap.add_argument("--corr-only", action="store_true", help="run only the correlation record")
    ap.add_argument("--agg-only", action="store_true", help="run only the soft-aggregation record")
    ap.add_argument("--vo-only", action="store_true", help="run only the sliding-window driver record")
    ap.add_argument("--vo-streams", type=int, default=256)
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--large-only", action="store_true",
                    help="run only the 64x256 large-window batch (for its profile) and print its record")
    ap.add_argument("--large-windows", type=int, default=8)
    ap.add_argument("--large-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--pmc-workload", action="store_true",
                    help="run only the calibration copy and the solves (for counter runs)")
    ap.add_argument("--pmc-target", default="assemble", choices=["assemble", "large", "corr", "agg"],
                    help="what --pmc-workload runs after the calibration copy")
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

    if args.corr_only:
        print(json.dumps(run_correlation(args, torch)), flush=True)
        return
    if args.agg_only:
        print(json.dumps(run_aggregation(args, torch)), flush=True)
        return
    if args.vo_only:
        print(json.dumps(run_driver(args, torch)), flush=True)
        print(json.dumps(run_stream_serving(args, torch)), flush=True)
        return
    # the CPU baseline runs first, in processes started before the GPU is used
    cpu = None if args.no_cpu_baseline else cpu_oracle_baseline(args.cpu_budget)

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
    bound, bound_note = assembly_bound()
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
        "roofline": {"bound": bound, "bound_evidence": bound_note, "kernel": "k_assemble",
                     "achieved": round(achieved, 3),
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
    # parity of the timed batch's own results: four windows against the oracle
    from oracle import ba_oracle as O
    pn, dn = poses_out.cpu().numpy(), depth_out.cpu().numpy()
    pairs = []
    for i in range(4):
        f0, f1 = batch.frame_off[i], batch.frame_off[i + 1]
        p0, p1 = batch.patch_off[i], batch.patch_off[i + 1]
        pr, dr = O.solve(windows[i])
        pairs.append((pn[f0:f1], dn[p0:p1], pr, dr))
    out["parity"] = {"method_scale": parity_record(pairs, "oracle dense FP64 solve, windows 0-3 of the timed batch")}
    solver.close()
    del batch, poses_out, depth_out
    torch.cuda.empty_cache()

    if not args.no_large:
        out["large_window"] = run_large(args, torch)
        out["parity"]["large_window"] = out["large_window"]["parity"]
        log(f"large windows: {out['large_window']}")
    if not args.no_serve:
        s = run_serving(args, torch)
        out["serving"] = s
        out["parity"]["serving"] = s["parity"]
        out["latency_ms"] = {"batched_p50": s["batched"].get("p50_ms"), "batched_p99": s["batched"].get("p99_ms"),
                             "plain_p50": s["plain"].get("p50_ms"), "plain_p99": s["plain"].get("p99_ms")}
    if not args.no_extra:
        out["plain_fp64"] = run_plain_fp64(args, torch)
        out["parity"]["plain_fp64"] = out["plain_fp64"]["parity"]
        log(f"plain fp64: {out['plain_fp64']}")
        out["backward"] = run_backward(args, torch)
        log(f"backward: {out['backward']}")
        out["correlation"] = run_correlation(args, torch)
        log(f"correlation: {out['correlation']}")
        out["aggregation"] = run_aggregation(args, torch)
        log(f"aggregation: {out['aggregation']}")
        out["driver"] = run_driver(args, torch)
        out["parity"]["driver"] = out["driver"]["fp64"]["parity_stream0"]
        log(f"driver: {out['driver']}")
        out["stream_serving"] = run_stream_serving(args, torch)
        log(f"stream serving: {out['stream_serving']}")
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
