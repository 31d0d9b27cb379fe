"""Python front end of the gfx950 bundle-adjustment library.

`Solver` owns a library handle; `Batch` holds one call's device buffers
(torch tensors on the GPU) and host offsets.  PyTorch provides device memory
and the stream only; the solve runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import native
from .native import BAConfig, BAError, BAProblem

PRECISIONS = {"fp64": native.BA_PREC_FP64, "fp32": native.BA_PREC_FP32}
SCHEDULES = {"auto": native.BA_SCHED_AUTO, "split": native.BA_SCHED_SPLIT,
             "fused": native.BA_SCHED_FUSED}


@dataclasses.dataclass
class Batch:
    """Device buffers of a batch of windows (layout of include/dpba.h)."""
    frame_off: np.ndarray      # host int64 [W+1]
    patch_off: np.ndarray
    edge_off: np.ndarray
    n_fixed: np.ndarray        # host int32 [W]
    intrinsics: np.ndarray     # host f64 [W,4]
    poses: torch.Tensor        # dev f64 [F,7]
    patches: torch.Tensor      # dev f64 [P,3]
    anchor: torch.Tensor       # dev int32 [P]
    kk: torch.Tensor           # dev int32 [E]
    jj: torch.Tensor           # dev int32 [E]
    targets: torch.Tensor      # dev f32/f64 [E,2]
    weights: torch.Tensor      # dev f32/f64 [E,2]

    @property
    def n_windows(self) -> int:
        return int(len(self.n_fixed))

    @property
    def totals(self):
        return int(self.frame_off[-1]), int(self.patch_off[-1]), int(self.edge_off[-1])


def make_batch(windows: Sequence, precision: str = "fp32", device="cuda") -> Batch:
    """Concatenate synth.Window-like objects into device buffers."""
    dt = torch.float32 if precision == "fp32" else torch.float64
    W = len(windows)
    fo = np.zeros(W + 1, np.int64)
    po = np.zeros(W + 1, np.int64)
    eo = np.zeros(W + 1, np.int64)
    for i, w in enumerate(windows):
        fo[i + 1] = fo[i] + w.poses.shape[0]
        po[i + 1] = po[i] + w.patches.shape[0]
        eo[i + 1] = eo[i] + w.kk.shape[0]

    def cat(arrs, dtype):
        if len(arrs) == 0:
            return np.zeros(0, dtype)
        return np.concatenate([np.asarray(a, dtype) for a in arrs], 0)

    to = lambda a, d: torch.as_tensor(a).to(device=device, dtype=d).contiguous()
    return Batch(
        frame_off=fo, patch_off=po, edge_off=eo,
        n_fixed=np.asarray([w.n_fixed for w in windows], np.int32),
        intrinsics=np.ascontiguousarray(np.stack([np.asarray(w.intrinsics, np.float64) for w in windows])
                                        if W else np.zeros((0, 4))),
        poses=to(cat([w.poses for w in windows], np.float64).reshape(-1, 7), torch.float64),
        patches=to(cat([w.patches for w in windows], np.float64).reshape(-1, 3), torch.float64),
        anchor=to(cat([w.anchor for w in windows], np.int32), torch.int32),
        kk=to(cat([w.kk for w in windows], np.int32), torch.int32),
        jj=to(cat([w.jj for w in windows], np.int32), torch.int32),
        targets=to(cat([w.targets for w in windows], np.float64).reshape(-1, 2), dt),
        weights=to(cat([w.weights for w in windows], np.float64).reshape(-1, 2), dt))


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None or t.numel() == 0 else ctypes.c_void_p(t.data_ptr())


def _host(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Solver:
    """A library handle with fixed capacities.

    precision: "fp32" (FP32 linearisation and assembly, FP64 Cholesky and
    back-substitution) or "fp64".  schedule: "auto", "split" (one launch per
    stage) or "fused" (one persistent launch).  chunk_frames: source frames
    per assembly workgroup of the split schedule, 0 = chosen per call."""

    def __init__(self, precision: str = "fp32", iterations: int = 2, lam: float = 1e-4,
                 z_min: float = 0.1, schedule: str = "auto", max_windows: int = 1,
                 max_frames_per_window: int = 22, max_frames: Optional[int] = None,
                 max_patches: int = 4096, max_edges: int = 65536, chunk_frames: int = 0):
        self.lib = native.lib()
        self.precision = precision
        cfg = BAConfig()
        cfg.precision = PRECISIONS[precision]
        cfg.iterations = iterations
        cfg.lambda_ = lam
        cfg.z_min = z_min
        cfg.schedule = SCHEDULES[schedule]
        cfg.max_windows = max_windows
        cfg.max_frames_per_window = max_frames_per_window
        cfg.max_frames = max_frames if max_frames is not None else max_windows * max_frames_per_window
        cfg.max_patches = max_patches
        cfg.max_edges = max_edges
        cfg.chunk_frames = chunk_frames
        self.cfg = cfg
        h = ctypes.c_void_p()
        r = self.lib.ba_create(ctypes.byref(cfg), ctypes.byref(h))
        if r != native.BA_OK:
            raise BAError(r, "ba_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.ba_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, r: int):
        if r != native.BA_OK:
            raise BAError(r, self.lib.ba_last_error(self.h).decode())

    def _problem(self, b: Batch, poses_out, depth_out) -> BAProblem:
        p = BAProblem()
        p.n_windows = b.n_windows
        self._keep = [np.ascontiguousarray(b.frame_off, np.int64), np.ascontiguousarray(b.patch_off, np.int64),
                      np.ascontiguousarray(b.edge_off, np.int64), np.ascontiguousarray(b.n_fixed, np.int32),
                      np.ascontiguousarray(b.intrinsics, np.float64)]
        p.frame_off, p.patch_off, p.edge_off, p.n_fixed, p.intrinsics = [_host(a) for a in self._keep]
        p.poses_in, p.patches_in = _ptr(b.poses), _ptr(b.patches)
        p.anchor, p.kk, p.jj = _ptr(b.anchor), _ptr(b.kk), _ptr(b.jj)
        p.targets, p.weights = _ptr(b.targets), _ptr(b.weights)
        p.poses_out, p.depth_out = _ptr(poses_out), _ptr(depth_out)
        return p

    def solve(self, b: Batch, poses_out: Optional[torch.Tensor] = None,
              depth_out: Optional[torch.Tensor] = None, stream: Optional[torch.cuda.Stream] = None):
        """Enqueue the solve on `stream` (default: torch's current stream).
        Returns (poses_out [F,7] f64, depth_out [P] f64) device tensors."""
        F, P, _ = b.totals
        dev = b.poses.device
        if poses_out is None:
            poses_out = torch.empty((F, 7), dtype=torch.float64, device=dev)
        if depth_out is None:
            depth_out = torch.empty((P,), dtype=torch.float64, device=dev)
        p = self._problem(b, poses_out, depth_out)
        s = (stream or torch.cuda.current_stream(dev)).cuda_stream
        self._check(self.lib.ba_solve(self.h, ctypes.byref(p), ctypes.c_void_p(s)))
        self._last_w = b.n_windows
        return poses_out, depth_out

    def prepare(self, p: BAProblem, stream: torch.cuda.Stream, n_windows: int):
        """ba_prepare: host checks and descriptor upload on `stream` for the
        problem struct `p` (whose host arrays the caller keeps alive)."""
        self._check(self.lib.ba_prepare(self.h, ctypes.byref(p), ctypes.c_void_p(stream.cuda_stream)))
        self._last_w = n_windows

    def launch(self, stream: torch.cuda.Stream):
        """ba_launch: the capacity-sized, capturable kernel sequence of the
        last prepared problem."""
        self._check(self.lib.ba_launch(self.h, ctypes.c_void_p(stream.cuda_stream)))

    def set_timing(self, enable: bool = True, stages=None):
        """Bracket the kernel launches of `stages` (names from native.STAGES;
        all when None) with events (ba_set_timing)."""
        if not enable:
            mask = 0
        elif stages is None:
            mask = (1 << len(native.STAGES)) - 1
        else:
            mask = 0
            for st in stages:
                mask |= 1 << native.STAGES.index(st)
        self._check(self.lib.ba_set_timing(self.h, mask))

    def kernel_times(self):
        """{stage: (total ms, launches)} since the previous call (waits for them)."""
        ms = (ctypes.c_double * len(native.STAGES))()
        n = (ctypes.c_int32 * len(native.STAGES))()
        self._check(self.lib.ba_kernel_times(self.h, ms, n))
        return {st: (float(ms[i]), int(n[i])) for i, st in enumerate(native.STAGES)}

    def status(self) -> np.ndarray:
        """Per-window BA_W_* bits of the last call (waits for its stream)."""
        out = np.zeros(int(self.cfg.max_windows), np.int32)
        self._check(self.lib.ba_status(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return out[:int(getattr(self, "_last_w", 0))]

    def reduced_system(self, b: Batch, window: int = 0, stream=None):
        """(S [n,n], s [n]) of `window` at the input state, from the GPU kernels."""
        N = int(b.frame_off[window + 1] - b.frame_off[window])
        n = 6 * (N - int(b.n_fixed[window]))
        dev = b.poses.device
        S = torch.zeros((n, n), dtype=torch.float64, device=dev)
        s = torch.zeros((n,), dtype=torch.float64, device=dev)
        F, P, _ = b.totals
        scratch_p = torch.empty((max(F, 1), 7), dtype=torch.float64, device=dev)
        scratch_d = torch.empty((max(P, 1),), dtype=torch.float64, device=dev)
        p = self._problem(b, scratch_p, scratch_d)
        st = (stream or torch.cuda.current_stream(dev)).cuda_stream
        self._check(self.lib.ba_debug_reduced_system(self.h, ctypes.byref(p), window,
                                                     _ptr(S), _ptr(s), ctypes.c_void_p(st)))
        return S, s


def capacities_for(windows: Sequence, slack: float = 1.0):
    """Capacities (keyword arguments of Solver) that fit `windows`."""
    return dict(max_windows=max(1, len(windows)),
                max_frames_per_window=max([w.poses.shape[0] for w in windows] + [1]),
                max_frames=max(1, sum(w.poses.shape[0] for w in windows)),
                max_patches=max(1, int(slack * sum(w.patches.shape[0] for w in windows))),
                max_edges=max(1, int(slack * sum(w.kk.shape[0] for w in windows))))


def _backward(self, b: Batch, grad_poses: torch.Tensor, grad_depth: torch.Tensor, stream=None):
    """Vector-Jacobian product of the solve with respect to targets and weights.
    grad_poses: [F,7] f64 cotangent of poses_out; grad_depth: [P] f64 cotangent of
    depth_out.  Returns (grad_targets, grad_weights), [E,2] in the dtype of targets."""
    F, P, E = b.totals
    dev = b.poses.device
    gp = grad_poses.to(device=dev, dtype=torch.float64).contiguous()
    gd = grad_depth.to(device=dev, dtype=torch.float64).contiguous()
    gt = torch.empty((E, 2), dtype=b.targets.dtype, device=dev)
    gw = torch.empty((E, 2), dtype=b.targets.dtype, device=dev)
    scratch_p = torch.empty((max(F, 1), 7), dtype=torch.float64, device=dev)
    scratch_d = torch.empty((max(P, 1),), dtype=torch.float64, device=dev)
    p = self._problem(b, scratch_p, scratch_d)
    st = (stream or torch.cuda.current_stream(dev)).cuda_stream
    self._check(self.lib.ba_backward(self.h, ctypes.byref(p), _ptr(gp), _ptr(gd), _ptr(gt), _ptr(gw),
                                     ctypes.c_void_p(st)))
    self._last_w = b.n_windows
    return gt, gw


Solver.backward = _backward


class BAFunction(torch.autograd.Function):
    """(targets, weights) -> (poses_out, depth_out) through the GPU solve, with
    the library's adjoint as backward.  The initial state and the graph are
    constants (`batch` supplies them).

    The solve and its adjoint run in the precision of `solver`.  An FP64
    solver gives gradients within 1e-4 (entry by entry) of FP64 central
    differences and within 1e-8 of the exact gradient: use one where the
    gradient's accuracy matters.  An FP32 solver differentiates its own FP32
    iterates: its vector-Jacobian products are within 1e-3 (in norm) of the
    FP64 ones, and a loss that sits near its minimum, such as pose errors to
    ground truth, also sees the FP32 forward state in its cotangent."""

    @staticmethod
    def forward(ctx, targets, weights, solver: Solver, batch: Batch):
        b = dataclasses.replace(batch, targets=targets.detach().contiguous(),
                                weights=weights.detach().contiguous())
        poses, depth = solver.solve(b)
        ctx.solver, ctx.batch = solver, b
        return poses, depth

    @staticmethod
    def backward(ctx, grad_poses, grad_depth):
        if grad_poses is None:
            grad_poses = torch.zeros((ctx.batch.totals[0], 7), dtype=torch.float64, device=ctx.batch.poses.device)
        if grad_depth is None:
            grad_depth = torch.zeros((ctx.batch.totals[1],), dtype=torch.float64, device=ctx.batch.poses.device)
        gt, gw = ctx.solver.backward(ctx.batch, grad_poses, grad_depth)
        return gt, gw, None, None


def solve_noalloc(b: Batch, precision: str = "fp32", iterations: int = 2, lam: float = 1e-4,
                  z_min: float = 0.1, schedule: str = "auto", chunk_frames: int = 0,
                  poses_out: Optional[torch.Tensor] = None, depth_out: Optional[torch.Tensor] = None,
                  status_out: Optional[torch.Tensor] = None, stream: Optional[torch.cuda.Stream] = None):
    """ba_solve_noalloc: the solve without a handle, its workspace carved from
    the library's static device array.  The output tensors must be supplied by
    a caller that cannot allocate; when None they are allocated here (argument
    marshalling only).  Returns (poses_out, depth_out, status_out [W] int32)."""
    lib = native.lib()
    cfg = BAConfig()
    cfg.precision = PRECISIONS[precision]
    cfg.iterations = iterations
    cfg.lambda_ = lam
    cfg.z_min = z_min
    cfg.schedule = SCHEDULES[schedule]
    cfg.chunk_frames = chunk_frames
    F, P, _ = b.totals
    dev = b.poses.device
    if poses_out is None:
        poses_out = torch.empty((F, 7), dtype=torch.float64, device=dev)
    if depth_out is None:
        depth_out = torch.empty((P,), dtype=torch.float64, device=dev)
    if status_out is None:
        status_out = torch.empty((max(b.n_windows, 1),), dtype=torch.int32, device=dev)
    keep = [np.ascontiguousarray(b.frame_off, np.int64), np.ascontiguousarray(b.patch_off, np.int64),
            np.ascontiguousarray(b.edge_off, np.int64), np.ascontiguousarray(b.n_fixed, np.int32),
            np.ascontiguousarray(b.intrinsics, np.float64)]
    p = BAProblem()
    p.n_windows = b.n_windows
    p.frame_off, p.patch_off, p.edge_off, p.n_fixed, p.intrinsics = [_host(a) for a in keep]
    p.poses_in, p.patches_in = _ptr(b.poses), _ptr(b.patches)
    p.anchor, p.kk, p.jj = _ptr(b.anchor), _ptr(b.kk), _ptr(b.jj)
    p.targets, p.weights = _ptr(b.targets), _ptr(b.weights)
    p.poses_out, p.depth_out = _ptr(poses_out), _ptr(depth_out)
    s = (stream or torch.cuda.current_stream(dev)).cuda_stream
    r = lib.ba_solve_noalloc(ctypes.byref(cfg), ctypes.byref(p), _ptr(status_out), ctypes.c_void_p(s))
    if r != native.BA_OK:
        raise BAError(r, "ba_solve_noalloc failed")
    return poses_out, depth_out, status_out
