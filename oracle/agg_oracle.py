"""FP64 CPU oracle of the soft aggregation of Deep Patch Visual Odometry
(Teed, Lipson, Deng, arXiv 2208.04726).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never calls it and
shares no code with it.

What it computes, plainly, in float64 with numpy (Sec. 3.1 "SoftMax
Aggregation", Eq. 5): for an edge e of the patch graph with neighbour set
N(e), the channel-wise aggregate

    psi( sum_{x in N(e)} sigma(x) * phi(x)  /  sum_{x in N(e)} sigma(x) )

of the hidden states x of the neighbours, where phi and psi are linear layers
and sigma is a linear layer followed by a sigmoid, in two instantiations
(Sec. 3.1): patch aggregation, where edges are neighbours when they share a
patch, and frame aggregation, where edges are neighbours when they share the
target frame and their patches share the source frame.

Readings taken where the paper is silent (each is listed in the design notes):
  * N(e) contains e itself: the neighbours of e are all edges with its key
    (patch k; or the pair (source frame of k, target frame j));
  * the three layers map the hidden dimension onto itself, y = W x + b with W
    stored [out, in].
"""
from __future__ import annotations

import numpy as np

PATCH, FRAME = 0, 1


def group_keys(mode: int, kk: np.ndarray, jj: np.ndarray, anchor: np.ndarray, n_frames: int) -> np.ndarray:
    """The key that defines N(e): the patch, or (source frame, target frame)."""
    if mode == PATCH:
        return np.asarray(kk, np.int64)
    return np.asarray(anchor, np.int64)[kk] * n_frames + np.asarray(jj, np.int64)


def soft_aggregate(mode, x, kk, jj, anchor, n_frames, w_gate, b_gate, w_val, b_val, w_out, b_out,
                   intermediates=False):
    """Eq. 5 for every edge.  x: [E, dim]; weights [dim, dim] (out, in);
    biases [dim].  Returns [E, dim] float64 (and, with intermediates=True, a
    dict of the per-edge and per-group values)."""
    x = np.asarray(x, np.float64)
    z = x @ np.asarray(w_gate, np.float64).T + np.asarray(b_gate, np.float64)
    f = x @ np.asarray(w_val, np.float64).T + np.asarray(b_val, np.float64)
    s = 1.0 / (1.0 + np.exp(-z))
    key = group_keys(mode, kk, jj, anchor, n_frames)
    uniq, inv = np.unique(key, return_inverse=True)
    G, D = len(uniq), x.shape[1]
    A = np.zeros((G, D))
    B = np.zeros((G, D))
    for e in range(x.shape[0]):
        A[inv[e]] += s[e] * f[e]
        B[inv[e]] += s[e]
    y = A / B
    o = y @ np.asarray(w_out, np.float64).T + np.asarray(b_out, np.float64)
    out = o[inv]
    if intermediates:
        return out, dict(z=z, f=f, s=s, group=inv, A=A, B=B, y=y, n=np.bincount(inv, minlength=G))
    return out
