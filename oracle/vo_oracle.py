"""Plain Python oracle of the sliding-window driver of Deep Patch Visual
Odometry (Teed, Lipson, Deng, arXiv 2208.04726), around the FP64 BA oracle.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never calls it and
shares no code with it.

Per new frame of a camera stream it applies, in this order, the rules of
Sec. 3.3 "VO System":

  * window advance: a window holds at most `window` keyframes; when it is
    full, the oldest keyframe leaves it with its patches and edges (its pose
    is final);
  * expansion: the new frame's pose by a constant-velocity motion model,
    T_n = (T_{n-1} T_{n-2}^-1) T_{n-1} ("Expansion"); its patches' inverse
    depth the median of all patches of the previous 3 keyframes; edges from
    every new patch to every keyframe within distance r of its frame, and
    from every patch of the last r keyframes to the new frame;
  * optimization: two Gauss-Newton iterations of the bundle adjustment with
    the poses of all but the last 10 keyframes fixed ("Optimization"), the
    targets and weights of the edges coming from the update operator (here a
    sensor table);
  * keyframing: the flow magnitude between keyframes t-5 and t-3; below the
    threshold (64 px) keyframe t-4 is removed and its pose relative to its
    previous neighbour stored ("Keyframing").

Readings taken where the paper is silent (each is listed in the design notes):
  * the first two frames of a stream take their poses from the
    initialisation, the first frame's patches a given inverse depth;
  * at least two poses stay fixed (the gauge), so n_fixed =
    max(min(2, n), n - 10) of n keyframes;
  * the flow magnitude is the mean, over the patches of keyframe t-5 whose
    homogeneous depth in keyframe t-3 exceeds 0.1, of the distance between
    a patch centre and its reprojection into keyframe t-3 (infinite when no
    patch qualifies);
  * the median of an even count is the mean of the two middle values.
"""
from __future__ import annotations

import types
from typing import Dict, List

import numpy as np
import torch

from oracle import ba_oracle as O


def _rt(pose):
    q = torch.as_tensor(pose[3:], dtype=O.DT)
    return O.quat_to_rot(q).numpy(), np.asarray(pose[:3], np.float64)


def _compose(a, b):
    """Pose 7-vector of T_a T_b."""
    qa, qb = torch.as_tensor(a[3:], dtype=O.DT), torch.as_tensor(b[3:], dtype=O.DT)
    Ra = O.quat_to_rot(qa).numpy()
    q = O.quat_mul(qa, qb).numpy()
    q = q / np.linalg.norm(q)
    return np.concatenate([Ra @ b[:3] + a[:3], q])


def _inverse(a):
    R, t = _rt(a)
    q = np.array([-a[3], -a[4], -a[5], a[6]])
    return np.concatenate([-R.T @ t, q])


def constant_velocity(p1, p2):
    """T_{n} = (T_{n-1} T_{n-2}^-1) T_{n-1} from p1 = T_{n-1}, p2 = T_{n-2}."""
    return _compose(_compose(p1, _inverse(p2)), p1)


def reproject(xy, d, pose_i, pose_j, intr):
    """Eq. 2 for patch centres: pixels in frame j and the homogeneous depth."""
    fx, fy, cx, cy = intr
    Ri, ti = _rt(pose_i)
    Rj, tj = _rt(pose_j)
    Rji = Rj @ Ri.T
    tji = tj - Rji @ ti
    ray = np.stack([(xy[:, 0] - cx) / fx, (xy[:, 1] - cy) / fy, np.ones(len(xy))], 1)
    p = ray @ Rji.T + d[:, None] * tji
    return np.stack([fx * p[:, 0] / p[:, 2] + cx, fy * p[:, 1] / p[:, 2] + cy], 1), p[:, 2]


class StreamOracle:
    def __init__(self, stream, window=22, radius=13, n_free=10, flow_thresh=64.0, z_min=0.1, iterations=2):
        self.s = stream
        self.N, self.r, self.n_free, self.thresh, self.z_min, self.K = window, radius, n_free, flow_thresh, z_min, \
            iterations
        self.ppf = stream.ppf
        self.kf: List[int] = []                 # frame id of each keyframe, in window order
        self.poses: List[np.ndarray] = []
        self.xy: List[np.ndarray] = []          # [ppf, 2] per keyframe
        self.depth: List[np.ndarray] = []       # [ppf] per keyframe
        self.edges: List[tuple] = []            # (patch id g = frame * ppf + i, frame id)
        self.final: Dict[int, np.ndarray] = {}  # frame id -> pose when it left the window
        self.removed: List[tuple] = []          # (frame id, previous keyframe id, relative pose)

    def _drop(self, pos):
        fid = self.kf[pos]
        self.edges = [(g, f) for (g, f) in self.edges if f != fid and g // self.ppf != fid]
        for lst in (self.kf, self.poses, self.xy, self.depth):
            del lst[pos]
        return fid

    def step(self, t):
        s, ppf = self.s, self.ppf
        if len(self.kf) == self.N:
            pose0 = self.poses[0]
            self.final[self._drop(0)] = pose0
        n = len(self.kf)
        pose = s.init_poses[n].copy() if n < 2 else constant_velocity(self.poses[n - 1], self.poses[n - 2])
        if n == 0:
            d = np.full(ppf, s.init_depth)
        else:
            d = np.full(ppf, float(np.median(np.concatenate(self.depth[max(0, n - 3):n]))))
        new_edges = []
        for p in range(max(0, n - self.r), n):
            new_edges += [(self.kf[p] * ppf + i, t) for i in range(ppf)]
        self.kf.append(t)
        self.poses.append(pose)
        self.xy.append(s.xy[t].copy())
        self.depth.append(d)
        for q in range(max(0, n - self.r), n + 1):
            new_edges += [(t * ppf + i, self.kf[q]) for i in range(ppf)]
        self.edges += new_edges
        n += 1
        # optimization
        pos = {f: i for i, f in enumerate(self.kf)}
        g = np.array([e[0] for e in self.edges])
        f = np.array([e[1] for e in self.edges])
        a = g // ppf
        o = f - a + s.R
        assert np.all((o >= 0) & (o <= 2 * s.R)), "edge beyond the sensor table"
        w = types.SimpleNamespace(
            poses=np.stack(self.poses),
            patches=np.concatenate([np.concatenate([self.xy[p], self.depth[p][:, None]], 1) for p in range(n)]),
            anchor=np.repeat(np.arange(n), ppf), kk=np.array([pos[x] * ppf + gi % ppf for x, gi in zip(a, g)]),
            jj=np.array([pos[x] for x in f]), targets=s.table_t[g, o], weights=s.table_w[g, o],
            intrinsics=s.intrinsics, n_fixed=max(min(2, n), n - self.n_free))
        poses, depth = O.solve(w, iterations=self.K, z_min=self.z_min)
        self.poses = [poses[p].copy() for p in range(n)]
        self.depth = [depth[p * ppf:(p + 1) * ppf].copy() for p in range(n)]
        # keyframing
        flow, removed = None, None
        if n >= 6:
            a_, b_ = n - 6, n - 4
            uv, Z = reproject(self.xy[a_], self.depth[a_], self.poses[a_], self.poses[b_], s.intrinsics)
            ok = Z > self.z_min
            flow = float(np.linalg.norm(uv[ok] - self.xy[a_][ok], axis=1).mean()) if ok.any() else float("inf")
            if flow < self.thresh:
                q = n - 5
                rel = _compose(self.poses[q], _inverse(self.poses[q - 1]))
                removed = (self.kf[q], self.kf[q - 1], rel)
                self.removed.append(removed)
                self._drop(q)
        return dict(kf=list(self.kf), edges=sorted(self.edges), flow=flow,
                    removed=None if removed is None else removed[0],
                    poses=np.stack(self.poses), depth=np.concatenate(self.depth))
