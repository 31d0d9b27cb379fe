"""Python front end of the gfx950 sliding-window driver (include/dpvo.h):
argument marshalling only; the driver's rules and the bundle adjustment run
in the library's HIP kernels, the streams' windows stay on the device."""
from __future__ import annotations

import ctypes
from typing import Sequence

import numpy as np
import torch

from . import native
from .native import BAError, VOConfig

PRECISIONS = {"fp64": native.BA_PREC_FP64, "fp32": native.BA_PREC_FP32}


def _host(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Driver:
    """Many camera streams stepped together.  `streams` supply the sensor
    tables (synth.Stream-like: table_t, table_w, xy, init_poses, init_depth,
    R, intrinsics)."""

    def __init__(self, streams: Sequence, precision: str = "fp64", window: int = 22, radius: int = 13,
                 n_free: int = 10, iterations: int = 2, flow_thresh: float = 64.0, lam: float = 1e-4,
                 z_min: float = 0.1, device="cuda"):
        self.lib = native.lib()
        self.streams = list(streams)
        s0 = self.streams[0]
        self.S, self.N, self.ppf = len(self.streams), window, s0.xy.shape[1]
        cfg = VOConfig()
        cfg.n_streams, cfg.window, cfg.patches_per_frame, cfg.radius = self.S, window, self.ppf, radius
        cfg.n_free, cfg.precision, cfg.iterations, cfg.table_radius = n_free, PRECISIONS[precision], iterations, s0.R
        cfg.flow_thresh, cfg.lambda_, cfg.z_min = flow_thresh, lam, z_min
        for i in range(4):
            cfg.intrinsics[i] = float(s0.intrinsics[i])
        h = ctypes.c_void_p()
        r = self.lib.vo_create(ctypes.byref(cfg), ctypes.byref(h))
        if r != native.BA_OK:
            raise BAError(r, "vo_create failed")
        self.h = h
        # sensor tables of all streams, concatenated on the device
        self.tab_t = torch.as_tensor(np.concatenate([s.table_t for s in self.streams]), device=device).contiguous()
        self.tab_w = torch.as_tensor(np.concatenate([s.table_w for s in self.streams]), device=device).contiguous()
        rows = np.array([s.table_t.shape[0] for s in self.streams], np.int64)
        self.tab_off = np.concatenate([[0], np.cumsum(rows)[:-1]]).astype(np.int64)
        self.tab_frames = np.array([s.poses_gt.shape[0] for s in self.streams], np.int32)
        self._check(self.lib.vo_set_sensor(self.h, ctypes.c_void_p(self.tab_t.data_ptr()),
                                           ctypes.c_void_p(self.tab_w.data_ptr()), _host(self.tab_off),
                                           _host(self.tab_frames)))
        self.init_poses = torch.as_tensor(np.stack([s.init_poses for s in self.streams]), device=device).contiguous()
        self.init_depth = np.array([s.init_depth for s in self.streams], np.float64)
        self.device = device

    def _check(self, r):
        if r != native.BA_OK:
            raise BAError(r, "sliding-window driver call failed")

    def step(self, frame_ids, stream=None):
        """One new frame per stream (frame_ids[s] < 0: stream idle)."""
        fid = np.ascontiguousarray(frame_ids, np.int32)
        xy = np.zeros((self.S, self.ppf, 2))
        for i, s in enumerate(self.streams):
            if fid[i] >= 0:
                xy[i] = s.xy[fid[i]]
        self._xy = torch.as_tensor(xy, device=self.device).contiguous()
        st = ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)
        self._check(self.lib.vo_step(self.h, _host(fid), ctypes.c_void_p(self._xy.data_ptr()),
                                     ctypes.c_void_p(self.init_poses.data_ptr()), _host(self.init_depth), st))

    def read(self):
        n = np.zeros(self.S, np.int32)
        ids = np.zeros((self.S, self.N), np.int32)
        flow = np.zeros(self.S, np.float64)
        rem = np.zeros(self.S, np.int32)
        self._check(self.lib.vo_read(self.h, _host(n), _host(ids), _host(flow), _host(rem)))
        return n, ids, flow, rem

    def window(self, s: int):
        poses = np.zeros((self.N, 7))
        depth = np.zeros(self.N * self.ppf)
        ne = ctypes.c_int64()
        self._check(self.lib.vo_read_window(self.h, s, None, None, None, None, ctypes.byref(ne)))
        g = np.zeros(max(ne.value, 1), np.int32)
        f = np.zeros(max(ne.value, 1), np.int32)
        self._check(self.lib.vo_read_window(self.h, s, _host(poses), _host(depth), _host(g), _host(f),
                                            ctypes.byref(ne)))
        return poses, depth, g[:ne.value], f[:ne.value]

    def status(self):
        out = np.zeros(self.S, np.int32)
        self._check(self.lib.vo_status(self.h, _host(out)))
        return out

    def close(self):
        if getattr(self, "h", None):
            self.lib.vo_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
