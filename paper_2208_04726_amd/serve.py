"""Batched serving of bundle-adjustment requests on one GPU.

A visual-odometry front end runs two BA iterations after every update of its
sliding window (Sec. 3.3 "Optimization"); a server that hosts many camera
streams receives one such window per update and per stream.  Windows are
independent, so the server packs whatever requests are waiting into one
batched solve:

  * slots: each slot owns a library handle, fixed device buffers sized for its
    capacities (windows, frames, patches, edges: the slot's HBM footprint),
    pinned host staging, a HIP stream and, optionally, a graph of the
    capacity-sized kernel sequence (ba_launch) captured once at start-up;
  * admission: requests are taken first-come first-served while the batch
    still fits the slot's footprint (continuous batching: a slot launches as
    soon as it is free and a request waits; a request never waits for a batch
    to fill); a request larger than a slot is answered at once with
    BA_E_CAPACITY; slots are created while the measured footprint of one
    slot still leaves a reserve of free HBM;
  * per batch: pack into pinned staging, one asynchronous copy per array,
    ba_prepare (descriptor upload) and the graph replay (or ba_launch), copies
    of the results back to pinned memory and an event; the host polls the
    events and hands each request its result.

`PlainServer` is the baseline: one ba_solve per request on one stream.

Every step of the solve runs in the library's HIP kernels; this module only
moves bytes and keeps the books.
"""
from __future__ import annotations

import collections
import contextlib
import ctypes
import dataclasses
import gc
import time
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import native
from .native import BAProblem
from .solver import Solver


@dataclasses.dataclass
class Request:
    """One window to solve (host arrays in the dtypes the library takes)."""
    rid: int
    stream: int                 # camera stream the window belongs to
    arrival: float              # seconds from the start of the trace
    n_fixed: int
    intrinsics: np.ndarray      # f64 [4]
    poses: np.ndarray           # f64 [N,7]
    patches: np.ndarray         # f64 [M,3]
    anchor: np.ndarray          # i32 [M]
    kk: np.ndarray              # i32 [E]
    jj: np.ndarray              # i32 [E]
    targets: np.ndarray         # f32/f64 [E,2]
    weights: np.ndarray         # f32/f64 [E,2]

    @property
    def shape(self):
        return self.poses.shape[0], self.patches.shape[0], self.kk.shape[0]


def request_from_window(w, rid: int = 0, stream: int = 0, arrival: float = 0.0,
                        precision: str = "fp32") -> Request:
    dt = np.float32 if precision == "fp32" else np.float64
    return Request(rid=rid, stream=stream, arrival=arrival, n_fixed=int(w.n_fixed),
                   intrinsics=np.asarray(w.intrinsics, np.float64).reshape(4),
                   poses=np.ascontiguousarray(w.poses, np.float64).reshape(-1, 7),
                   patches=np.ascontiguousarray(w.patches, np.float64).reshape(-1, 3),
                   anchor=np.ascontiguousarray(w.anchor, np.int32),
                   kk=np.ascontiguousarray(w.kk, np.int32),
                   jj=np.ascontiguousarray(w.jj, np.int32),
                   targets=np.ascontiguousarray(w.targets, dt).reshape(-1, 2),
                   weights=np.ascontiguousarray(w.weights, dt).reshape(-1, 2))


@dataclasses.dataclass(frozen=True)
class Capacity:
    """What one batched solve may hold (the slot's footprint)."""
    windows: int
    frames: int
    patches: int
    edges: int
    frames_per_window: int = 22

    def fits(self, r: Request) -> bool:
        N, M, E = r.shape
        return (N <= self.frames_per_window and N <= self.frames and M <= self.patches
                and E <= self.edges)


def admit(pending: "collections.deque[Request]", cap: Capacity) -> List[Request]:
    """Take requests from the head of `pending` while the batch fits `cap`
    (first come, first served; stops at the first request that does not fit).
    A request that can never fit a slot must be rejected before it is queued."""
    batch: List[Request] = []
    F = P = E = 0
    while pending and len(batch) < cap.windows:
        r = pending[0]
        N, M, Ee = r.shape
        if F + N > cap.frames or P + M > cap.patches or E + Ee > cap.edges:
            break
        batch.append(pending.popleft())
        F, P, E = F + N, P + M, E + Ee
    return batch


def _pinned(shape, dtype):
    return torch.empty(shape, dtype=dtype, pin_memory=True)


class _Buffers:
    """Device buffers plus pinned host staging of one batch of capacity `cap`."""

    def __init__(self, cap: Capacity, precision: str, device):
        dt = torch.float32 if precision == "fp32" else torch.float64
        F, P, E = cap.frames, max(cap.patches, 1), max(cap.edges, 1)
        spec = {"poses": ((F, 7), torch.float64), "patches": ((P, 3), torch.float64),
                "anchor": ((P,), torch.int32), "kk": ((E,), torch.int32), "jj": ((E,), torch.int32),
                "targets": ((E, 2), dt), "weights": ((E, 2), dt)}
        self.dev = {k: torch.empty(s, dtype=d, device=device) for k, (s, d) in spec.items()}
        self.host = {k: _pinned(s, d) for k, (s, d) in spec.items()}
        self.hnp = {k: v.numpy() for k, v in self.host.items()}
        self.poses_out = torch.empty((F, 7), dtype=torch.float64, device=device)
        self.depth_out = torch.empty((P,), dtype=torch.float64, device=device)
        self.h_poses_out = _pinned((F, 7), torch.float64)
        self.h_depth_out = _pinned((P,), torch.float64)
        W = cap.windows
        self.frame_off = np.zeros(W + 1, np.int64)
        self.patch_off = np.zeros(W + 1, np.int64)
        self.edge_off = np.zeros(W + 1, np.int64)
        self.n_fixed = np.zeros(W, np.int32)
        self.intr = np.zeros((W, 4), np.float64)
        p = BAProblem()
        host = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        devp = lambda t: ctypes.c_void_p(t.data_ptr())
        p.frame_off, p.patch_off, p.edge_off = host(self.frame_off), host(self.patch_off), host(self.edge_off)
        p.n_fixed, p.intrinsics = host(self.n_fixed), host(self.intr)
        p.poses_in, p.patches_in = devp(self.dev["poses"]), devp(self.dev["patches"])
        p.anchor, p.kk, p.jj = devp(self.dev["anchor"]), devp(self.dev["kk"]), devp(self.dev["jj"])
        p.targets, p.weights = devp(self.dev["targets"]), devp(self.dev["weights"])
        p.poses_out, p.depth_out = devp(self.poses_out), devp(self.depth_out)
        p.n_windows = 0
        self.problem = p

    def pack(self, batch: Sequence[Request]):
        """Write the batch into pinned staging; returns the totals (F, P, E)."""
        F = P = E = 0
        h = self.hnp
        for i, r in enumerate(batch):
            N, M, Ee = r.shape
            h["poses"][F:F + N] = r.poses
            h["patches"][P:P + M] = r.patches
            h["anchor"][P:P + M] = r.anchor
            h["kk"][E:E + Ee] = r.kk
            h["jj"][E:E + Ee] = r.jj
            h["targets"][E:E + Ee] = r.targets
            h["weights"][E:E + Ee] = r.weights
            self.n_fixed[i] = r.n_fixed
            self.intr[i] = r.intrinsics
            F, P, E = F + N, P + M, E + Ee
            self.frame_off[i + 1], self.patch_off[i + 1], self.edge_off[i + 1] = F, P, E
        self.problem.n_windows = len(batch)
        return F, P, E

    def upload(self, F: int, P: int, E: int):
        """Asynchronous host-to-device copies on the current stream."""
        rows = {"poses": F, "patches": P, "anchor": P, "kk": E, "jj": E, "targets": E, "weights": E}
        for k, n in rows.items():
            if n:
                self.dev[k][:n].copy_(self.host[k][:n], non_blocking=True)

    def download(self, F: int, P: int):
        if F:
            self.h_poses_out[:F].copy_(self.poses_out[:F], non_blocking=True)
        if P:
            self.h_depth_out[:P].copy_(self.depth_out[:P], non_blocking=True)


@dataclasses.dataclass
class Result:
    rid: int
    poses: np.ndarray      # f64 [N,7]
    depth: np.ndarray      # f64 [M]
    status: int            # BA_W_* bits, or BA_E_CAPACITY for a request no slot can hold
    latency: float         # seconds, arrival to result on the host


def rejected(r: Request, latency: float = 0.0) -> Result:
    """The answer to a request larger than a slot: BA_E_CAPACITY, the inputs
    unchanged."""
    return Result(r.rid, r.poses.copy(), r.patches[:, 2].copy(), native.BA_E_CAPACITY, latency)


class _Slot:
    def __init__(self, cap: Capacity, precision: str, iterations: int, schedule: str,
                 chunk_frames: int, use_graph: bool, device):
        self.cap = cap
        self.solver = Solver(precision=precision, iterations=iterations, schedule=schedule,
                             max_windows=cap.windows, max_frames_per_window=cap.frames_per_window,
                             max_frames=cap.frames, max_patches=max(cap.patches, 1),
                             max_edges=max(cap.edges, 1), chunk_frames=chunk_frames)
        self.buf = _Buffers(cap, precision, device)
        self.stream = torch.cuda.Stream(device=device)
        self.event = torch.cuda.Event()
        self.batch: List[Request] = []
        self.totals = (0, 0, 0)
        self.graph = None
        if use_graph:
            # capture the capacity-sized kernel sequence once; an empty batch is
            # prepared first so that the captured launches see this slot's buffers
            self.solver.prepare(self.buf.problem, self.stream, 0)
            self.stream.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=self.stream):
                self.solver.launch(torch.cuda.current_stream())
            self.graph = g
            self.stream.synchronize()

    @property
    def busy(self) -> bool:
        return bool(self.batch)

    def launch(self, batch: List[Request]):
        F, P, E = self.buf.pack(batch)
        self.batch, self.totals = batch, (F, P, E)
        with torch.cuda.stream(self.stream):
            self.buf.upload(F, P, E)
            self.solver.prepare(self.buf.problem, self.stream, len(batch))
            if self.graph is not None:
                self.graph.replay()
            else:
                self.solver.launch(self.stream)
            self.buf.download(F, P)
            self.event.record(self.stream)

    def done(self) -> bool:
        return self.event.query()

    def collect(self, t_now: float) -> List[Result]:
        """Results of the finished batch (the stream has passed the event)."""
        status = self.solver.status()
        out = []
        F = P = 0
        hp, hd = self.buf.h_poses_out.numpy(), self.buf.h_depth_out.numpy()
        for i, r in enumerate(self.batch):
            N, M, _ = r.shape
            out.append(Result(r.rid, hp[F:F + N].copy(), hd[P:P + M].copy(), int(status[i]),
                              t_now - r.arrival))
            F, P = F + N, P + M
        self.batch = []
        return out


@contextlib.contextmanager
def _no_gc():
    """The serving loops keep Python's cyclic garbage collector off: a full
    collection over the results gathered so far stalls the loop for tens of
    milliseconds."""
    was = gc.isenabled()
    gc.disable()
    try:
        yield
    finally:
        if was:
            gc.enable()


class BatchedServer:
    """Continuous batching over `n_slots` slots of capacity `cap`.

    schedule: "fused" (one persistent launch per batch) or "split"; with
    "split", chunk_frames > 0 keeps each window's arithmetic independent of
    the rest of its batch (the fused schedule always does)."""

    def __init__(self, cap: Capacity, n_slots: int = 2, precision: str = "fp32",
                 iterations: int = 2, schedule: str = "fused", chunk_frames: int = 11,
                 use_graph: bool = True, device="cuda", hbm_reserve: float = 0.1):
        if schedule not in ("fused", "split"):
            raise ValueError("schedule must be 'fused' or 'split'")
        self.cap = cap
        total = torch.cuda.mem_get_info(device)[1]
        free0 = torch.cuda.mem_get_info(device)[0]
        # slots are admitted by HBM footprint: the first slot's footprint is
        # measured, and further slots are created while the free HBM after
        # them stays above `hbm_reserve` of the device
        self.slots = [_Slot(cap, precision, iterations, schedule, chunk_frames, use_graph, device)]
        torch.cuda.synchronize(device)
        self.slot_bytes = int(free0 - torch.cuda.mem_get_info(device)[0])
        while len(self.slots) < n_slots:
            free = torch.cuda.mem_get_info(device)[0]
            if free - self.slot_bytes < hbm_reserve * total:
                break
            self.slots.append(_Slot(cap, precision, iterations, schedule, chunk_frames, use_graph, device))
        torch.cuda.synchronize(device)
        # device memory the slots hold (buffers, library workspace, graphs)
        self.footprint_bytes = int(free0 - torch.cuda.mem_get_info(device)[0])
        self.batches = 0
        self.batch_sizes: List[int] = []

    def run(self, requests: Sequence[Request], clock=time.perf_counter) -> Dict[int, Result]:
        """Serve `requests` (sorted by arrival) in real time: a request becomes
        visible at its arrival time.  A request no slot can hold is answered at
        its arrival with BA_E_CAPACITY (`rejected`); the others are served.
        Returns rid -> Result."""
        with _no_gc():
            return self._run(requests, clock)

    def _run(self, requests: Sequence[Request], clock) -> Dict[int, Result]:
        pending: "collections.deque[Request]" = collections.deque()
        results: Dict[int, Result] = {}
        n = len(requests)
        i = 0
        t0 = clock()
        while len(results) < n:
            now = clock() - t0
            while i < n and requests[i].arrival <= now:
                r = requests[i]
                if self.cap.fits(r):
                    pending.append(r)
                else:
                    results[r.rid] = rejected(r, clock() - t0 - r.arrival)
                i += 1
            for s in self.slots:
                if s.busy and s.done():
                    for res in s.collect(clock() - t0):
                        results[res.rid] = res
            if pending:
                for s in self.slots:
                    if not s.busy and pending:
                        batch = admit(pending, self.cap)
                        s.launch(batch)
                        self.batches += 1
                        self.batch_sizes.append(len(batch))
        return results


class PlainServer:
    """Baseline: one ba_solve per request, in arrival order, on one stream."""

    def __init__(self, cap: Capacity, precision: str = "fp32", iterations: int = 2,
                 schedule: str = "split", device="cuda"):
        one = Capacity(1, cap.frames_per_window, cap.patches, cap.edges, cap.frames_per_window)
        self.cap = one
        self.solver = Solver(precision=precision, iterations=iterations, schedule=schedule,
                             max_windows=1, max_frames_per_window=cap.frames_per_window,
                             max_frames=cap.frames_per_window, max_patches=max(cap.patches, 1),
                             max_edges=max(cap.edges, 1))
        self.buf = _Buffers(one, precision, device)
        self.stream = torch.cuda.Stream(device=device)

    def run(self, requests: Sequence[Request], clock=time.perf_counter) -> Dict[int, Result]:
        with _no_gc():
            return self._run(requests, clock)

    def _run(self, requests: Sequence[Request], clock) -> Dict[int, Result]:
        results: Dict[int, Result] = {}
        lib, h = self.solver.lib, self.solver.h
        t0 = clock()
        for r in requests:
            while clock() - t0 < r.arrival:
                pass
            if not self.cap.fits(r):
                results[r.rid] = rejected(r, clock() - t0 - r.arrival)
                continue
            F, P, E = self.buf.pack([r])
            with torch.cuda.stream(self.stream):
                self.buf.upload(F, P, E)
                rc = lib.ba_solve(h, ctypes.byref(self.buf.problem), ctypes.c_void_p(self.stream.cuda_stream))
                if rc != native.BA_OK:
                    raise native.BAError(rc, lib.ba_last_error(h).decode())
                self.buf.download(F, P)
            self.stream.synchronize()
            self.solver._last_w = 1
            st = int(self.solver.status()[0])
            results[r.rid] = Result(r.rid, self.buf.h_poses_out.numpy()[:F].copy(),
                                    self.buf.h_depth_out.numpy()[:P].copy(), st, clock() - t0 - r.arrival)
        return results


def poisson_trace(pool: Sequence[Request], n: int, rate: float, n_streams: int = 64,
                  seed: int = 0) -> List[Request]:
    """n requests with exponential inter-arrival times at `rate` per second,
    each a window drawn uniformly from `pool`, stream id uniform in
    [0, n_streams).  rate = inf gives a closed batch (all arrive at 0)."""
    rng = np.random.default_rng(seed)
    if np.isinf(rate):
        t = np.zeros(n)
    else:
        t = np.cumsum(rng.exponential(1.0 / rate, n))
    pick = rng.integers(0, len(pool), n)
    sid = rng.integers(0, n_streams, n)
    return [dataclasses.replace(pool[int(pick[i])], rid=i, stream=int(sid[i]), arrival=float(t[i]))
            for i in range(n)]


def latency_summary(results: Dict[int, Result], skip: int = 0) -> Dict[str, float]:
    """p50 / p99 / p99.9 / mean latency in ms over requests with rid >= skip."""
    lat = np.array([r.latency for rid, r in results.items() if rid >= skip]) * 1e3
    if lat.size == 0:
        return {}
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "p999_ms": float(np.percentile(lat, 99.9)), "mean_ms": float(lat.mean()),
            "n": int(lat.size)}


# ---------------------------------------------------------------------------
# Stateful serving of camera streams on the sliding-window driver

@dataclasses.dataclass
class FrameRequest:
    rid: int
    stream: int
    frame: int
    arrival: float          # seconds after the start of the run


@dataclasses.dataclass
class FrameResult:
    rid: int
    stream: int
    frame: int
    latency: float          # seconds, arrival to the end of the step that took the frame
    batch: int              # frames stepped together with this one (itself included)


def frame_trace(n_streams: int, n_frames: int, fps: float, seed: int = 0,
                jitter: float = 0.1) -> List[FrameRequest]:
    """Every stream sends frames 0 .. n_frames-1 at `fps`, from a random phase
    in [0, 1/fps), each arrival jittered by up to `jitter` of a frame period;
    requests in arrival order (rid = position)."""
    rng = np.random.default_rng(seed)
    period = 1.0 / fps
    phase = rng.uniform(0, period, n_streams)
    reqs = []
    for s in range(n_streams):
        t = phase[s] + period * (np.arange(n_frames) + jitter * rng.uniform(0, 1, n_frames))
        reqs += [(float(t[f]), s, f) for f in range(n_frames)]
    reqs.sort()
    return [FrameRequest(i, s, f, t) for i, (t, s, f) in enumerate(reqs)]


def _wait_until(clock, t0, t):
    while clock() - t0 < t:
        dt = t - (clock() - t0)
        if dt > 2e-4:
            time.sleep(dt - 1e-4)


class StreamServer:
    """Continuous batching of camera streams whose windows live on the device
    (include/dpvo.h): every step takes the oldest waiting frame of every
    stream that has one and steps them together in one vo_step; a frame that
    arrives during a step joins the next one.  A stream's frames are stepped
    in order, one per step; nothing of a window is uploaded or read back."""

    def __init__(self, driver):
        self.driver = driver

    def run(self, requests: Sequence[FrameRequest], clock=time.perf_counter) -> Dict[int, FrameResult]:
        with _no_gc():
            return self._run(requests, clock)

    def _run(self, requests, clock):
        S = self.driver.S
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending = [collections.deque() for _ in range(S)]
        results: Dict[int, FrameResult] = {}
        fid = np.full(S, -1, np.int32)
        i, n = 0, len(reqs)
        t0 = clock()
        while len(results) < n:
            now = clock() - t0
            while i < n and reqs[i].arrival <= now:
                pending[reqs[i].stream].append(reqs[i])
                i += 1
            ready = [s for s in range(S) if pending[s]]
            if not ready:
                _wait_until(clock, t0, reqs[i].arrival)
                continue
            fid[:] = -1
            for s in ready:
                fid[s] = pending[s][0].frame
            self.driver.step(fid)
            t = clock() - t0
            for s in ready:
                r = pending[s].popleft()
                results[r.rid] = FrameResult(r.rid, r.stream, r.frame, t - r.arrival, len(ready))
        return results


class PlainStreamServer:
    """The baseline: one driver per stream and one frame per step, in arrival
    order."""

    def __init__(self, drivers):
        self.drivers = drivers

    def run(self, requests: Sequence[FrameRequest], clock=time.perf_counter) -> Dict[int, FrameResult]:
        with _no_gc():
            return self._run(requests, clock)

    def _run(self, requests, clock):
        reqs = sorted(requests, key=lambda r: r.arrival)
        one = np.zeros(1, np.int32)
        results: Dict[int, FrameResult] = {}
        t0 = clock()
        for r in reqs:
            _wait_until(clock, t0, r.arrival)
            one[0] = r.frame
            self.drivers[r.stream].step(one)
            results[r.rid] = FrameResult(r.rid, r.stream, r.frame, clock() - t0 - r.arrival, 1)
        return results


def frame_latency_summary(results: Dict[int, FrameResult], min_frame: int = 0) -> Dict[str, float]:
    """Latency percentiles (ms) over frames >= min_frame, the mean batch, and
    the frames per second the run sustained."""
    sel = [r for r in results.values() if r.frame >= min_frame]
    if not sel:
        return {}
    lat = np.array([r.latency for r in sel]) * 1e3
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
            "mean_batch": float(np.mean([r.batch for r in sel])), "n": len(sel)}
