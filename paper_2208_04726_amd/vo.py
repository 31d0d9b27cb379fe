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


def _quat_mul(a, b):
    ax, ay, az, aw = a
    bx, by, bz, bw = b
    return np.array([aw * bx + bw * ax + ay * bz - az * by, aw * by + bw * ay + az * bx - ax * bz,
                     aw * bz + bw * az + ax * by - ay * bx, aw * bw - ax * bx - ay * by - az * bz])


def _rot(q):
    x, y, z, w = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def compose(a, b):
    """Pose 7-vector (t, q) of T_a T_b."""
    q = _quat_mul(a[3:], b[3:])
    return np.concatenate([_rot(a[3:]) @ b[:3] + a[:3], q / np.linalg.norm(q)])


def assemble_trajectory(kf_ids, kf_poses, retired, removed):
    """Whole trajectory of a stream ("Keyframing", Sec. 3.3): keyframes in the
    window as they stand, keyframes that left full windows as they left
    (retired: frame id -> pose), and removed keyframes (removed: frame id ->
    (previous keyframe id, T_removed T_prev^-1)) as their relative pose
    applied to the pose of the keyframe before them, itself resolved the same
    way.  Returns frame id -> pose, in frame order."""
    out = {int(f): np.asarray(p) for f, p in zip(kf_ids, kf_poses)}
    out.update({int(f): np.asarray(p) for f, p in retired.items()})
    todo = sorted(f for f in removed if f not in out)
    while todo:
        left = []
        for f in todo:
            prev, rel = removed[f]
            if prev in out:
                out[f] = compose(rel, out[prev])
            else:
                left.append(f)
        if len(left) == len(todo):
            raise ValueError(f"removed keyframes {left} refer to frames never seen")
        todo = left
    return dict(sorted(out.items()))


def _host(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Driver:
    """Many camera streams stepped together.  `streams` supply the sensor
    tables (synth.Stream-like: table_t, table_w, xy, init_poses, init_depth,
    R, intrinsics)."""

    def __init__(self, streams: Sequence, precision: str = "fp64", window: int = 22, radius: int = 13,
                 n_free: int = 10, iterations: int = 2, flow_thresh: float = 64.0, lam: float = 1e-4,
                 z_min: float = 0.1, device="cuda", track_trajectory: bool = True):
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
        # sensor tables on the device, one copy per distinct stream object
        # (streams given more than once share their rows)
        uniq, where = [], {}
        for st_ in self.streams:
            if id(st_) not in where:
                where[id(st_)] = len(uniq)
                uniq.append(st_)
        rows = np.array([u.table_t.shape[0] for u in uniq], np.int64)
        first = np.concatenate([[0], np.cumsum(rows)[:-1]]).astype(np.int64)
        self.tab_t = torch.as_tensor(np.concatenate([u.table_t for u in uniq]), device=device).contiguous()
        self.tab_w = torch.as_tensor(np.concatenate([u.table_w for u in uniq]), device=device).contiguous()
        self.tab_off = np.array([first[where[id(st_)]] for st_ in self.streams], np.int64)
        self.tab_frames = np.array([s.poses_gt.shape[0] for s in self.streams], np.int32)
        self._check(self.lib.vo_set_sensor(self.h, ctypes.c_void_p(self.tab_t.data_ptr()),
                                           ctypes.c_void_p(self.tab_w.data_ptr()), _host(self.tab_off),
                                           _host(self.tab_frames)))
        self.init_poses = torch.as_tensor(np.stack([s.init_poses for s in self.streams]), device=device).contiguous()
        self.init_depth = np.array([s.init_depth for s in self.streams], np.float64)
        self.device = device
        # the new frames' patch centres: gathered on the host into pinned
        # memory, one asynchronous copy per step (vo_step waits for the step,
        # so the buffers are free again when it returns)
        self._uniq_xy = [u.xy for u in uniq]
        same = len({u.xy.shape for u in uniq}) == 1
        self._xy_all = np.stack(self._uniq_xy) if same else None
        self._which = np.array([where[id(st_)] for st_ in self.streams])
        self._xy_host = torch.zeros((self.S, self.ppf, 2), dtype=torch.float64, pin_memory=True)
        self._xy_dev = torch.zeros((self.S, self.ppf, 2), dtype=torch.float64, device=device)
        # per stream: final poses of keyframes that left full windows, and the
        # removed keyframes with their previous keyframe and relative pose
        self.track = track_trajectory
        self.retired = [dict() for _ in range(self.S)]
        self.removed = [dict() for _ in range(self.S)]

    def _check(self, r):
        if r != native.BA_OK:
            raise BAError(r, "sliding-window driver call failed")

    def step(self, frame_ids, stream=None):
        """One new frame per stream (frame_ids[s] < 0: stream idle)."""
        fid = np.ascontiguousarray(frame_ids, np.int32)
        if fid.shape != (self.S,):
            raise ValueError(f"frame_ids must have shape ({self.S},)")
        xy = self._xy_host.numpy()
        act = np.nonzero(fid >= 0)[0]
        if self._xy_all is not None:
            xy[act] = self._xy_all[self._which[act], fid[act]]
        else:
            for i in act:
                xy[i] = self._uniq_xy[self._which[i]][fid[i]]
        torch_stream = stream or torch.cuda.current_stream()
        with torch.cuda.stream(torch_stream):
            self._xy_dev.copy_(self._xy_host, non_blocking=True)
        st = ctypes.c_void_p(torch_stream.cuda_stream)
        self._check(self.lib.vo_step(self.h, _host(fid), ctypes.c_void_p(self._xy_dev.data_ptr()),
                                     ctypes.c_void_p(self.init_poses.data_ptr()), _host(self.init_depth), st))
        if self.track:
            ev = self.events()
            for i in range(self.S):
                if ev["retired"][i] >= 0:
                    self.retired[i][int(ev["retired"][i])] = ev["retired_pose"][i].copy()
                if ev["removed"][i] >= 0:
                    self.removed[i][int(ev["removed"][i])] = (int(ev["removed_prev"][i]), ev["removed_rel"][i].copy())

    def events(self):
        """What the last step took out of each window (vo_read_events)."""
        ev = dict(retired=np.zeros(self.S, np.int32), retired_pose=np.zeros((self.S, 7)),
                  removed=np.zeros(self.S, np.int32), removed_prev=np.zeros(self.S, np.int32),
                  removed_rel=np.zeros((self.S, 7)))
        self._check(self.lib.vo_read_events(self.h, _host(ev["retired"]), _host(ev["retired_pose"]),
                                            _host(ev["removed"]), _host(ev["removed_prev"]),
                                            _host(ev["removed_rel"])))
        return ev

    def trajectory(self, s: int):
        """Pose of every frame stream s has processed (assemble_trajectory)."""
        n, kf, _, _ = self.read()
        poses, _, _, _ = self.window(s)
        k = int(n[s])
        return assemble_trajectory(kf[s, :k].tolist(), poses[:k], self.retired[s], self.removed[s])

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
