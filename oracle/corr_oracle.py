"""FP64 CPU oracle of the correlation features of Deep Patch Visual Odometry
(Teed, Lipson, Deng, arXiv 2208.04726).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never calls it and
shares no code with it.

What it computes, plainly and slowly, in float64 with numpy:

  * the two-level matching-feature pyramid: the second level is the first
    averaged over s x s blocks with stride s (Sec. 3 "Feature and Patch
    Extraction": average pooling with a 4 x 4 filter and stride 4);
  * for every edge (k, j) of the patch graph and every pixel (u, v) of patch
    k, the inner products of the patch feature g_uv with the frame-j features
    bilinearly sampled on a 7 x 7 integer grid centred at the pixel's
    reprojection P'_kj(u, v) (Sec. 3.1 "Correlation", Eq. 4), at both pyramid
    levels, concatenated (Sec. 3.1; Appendix "Correlation Operation").

Readings taken where the paper is silent (each is listed in the design notes):
  * feature maps are indexed [frame, row y, column x, channel]; integer
    coordinates are pixel centres; bilinear sampling treats every pixel
    outside the map as a zero feature (zero padding);
  * the reprojected coordinates are given in pixels of the first pyramid
    level; level l samples at those coordinates divided by its scale s_l
    (s_0 = 1, s_1 = the pooling stride);
  * the grid offset of output (alpha, beta) is (dy, dx) = (alpha - 3, beta - 3):
    alpha runs over rows, beta over columns;
  * the output of an edge is [level, pixel u*p+v, alpha, beta].
"""
from __future__ import annotations

import numpy as np

RADIUS = 3                  # 7 x 7 grid (Sec. 3.1, Eq. 4)
GRID = 2 * RADIUS + 1


def avg_pool(fmap: np.ndarray, s: int) -> np.ndarray:
    """[F, H, W, D] -> [F, H // s, W // s, D]: mean of each s x s block
    (rows and columns beyond the last whole block are dropped)."""
    F, H, W, D = fmap.shape
    h, w = H // s, W // s
    out = np.zeros((F, h, w, D))
    for dy in range(s):
        for dx in range(s):
            out += fmap[:, dy:dy + h * s:s, dx:dx + w * s:s, :].astype(np.float64)
    return out / (s * s)


def bilinear(fmap: np.ndarray, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Bilinear samples of one frame's map [H, W, D] at points (x, y) of any
    shape; pixels outside the map count as zero features.  Returns
    [..., D] in float64."""
    H, W, D = fmap.shape
    x0 = np.floor(x).astype(np.int64)
    y0 = np.floor(y).astype(np.int64)
    fx, fy = x - x0, y - y0
    out = np.zeros(x.shape + (D,))
    for cy, wy in ((0, 1.0 - fy), (1, fy)):
        for cx, wx in ((0, 1.0 - fx), (1, fx)):
            yy, xx = y0 + cy, x0 + cx
            inside = (yy >= 0) & (yy < H) & (xx >= 0) & (xx < W)
            val = fmap[np.clip(yy, 0, H - 1), np.clip(xx, 0, W - 1)].astype(np.float64)
            out += (wy * wx * inside)[..., None] * val
    return out


def correlation(levels, scales, gmap: np.ndarray, coords: np.ndarray, kk: np.ndarray,
                jj: np.ndarray) -> np.ndarray:
    """Eq. 4 at every pyramid level.

    levels: list of [F, H_l, W_l, D] frame feature maps; scales: the divisor of
    the level-0 coordinates at each level; gmap: [M, p*p, D] patch features;
    coords: [E, p*p, 2] reprojected pixel (x, y) of every patch pixel, in
    level-0 pixels; kk, jj: [E] patch and target frame of each edge.
    Returns [E, n_levels, p*p, 7, 7] float64."""
    E, P2, _ = coords.shape
    off = np.arange(GRID) - RADIUS
    out = np.zeros((E, len(levels), P2, GRID, GRID))
    for e in range(E):
        g = gmap[kk[e]].astype(np.float64)                       # [p*p, D]
        for l, (fm, s) in enumerate(zip(levels, scales)):
            x = coords[e, :, 0].astype(np.float64) / s           # [p*p]
            y = coords[e, :, 1].astype(np.float64) / s
            gx = x[:, None, None] + off[None, None, :]           # [p*p, 7(alpha), 7(beta)]
            gy = y[:, None, None] + off[None, :, None]
            gx, gy = np.broadcast_arrays(gx, gy)
            f = bilinear(fm[jj[e]], gx, gy)                      # [p*p, 7, 7, D]
            out[e, l] = np.einsum("pabd,pd->pab", f, g)
    return out


def correlation_abs(levels, scales, gmap, coords, kk, jj) -> np.ndarray:
    """Eq. 4 with every term replaced by its absolute value: the summed
    magnitudes that bound the rounding error of any evaluation order."""
    return correlation([np.abs(f) for f in levels], scales, np.abs(gmap), coords, kk, jj)
