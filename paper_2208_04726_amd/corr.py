"""Python front end of the gfx950 correlation features (include/dpcorr.h):
argument marshalling only, every step runs in the library's HIP kernels.
Feature tensors are torch.bfloat16 on the GPU, channels last."""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import native
from .native import BAError, DPCProblem


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(t: torch.Tensor, stream):
    return ctypes.c_void_p((stream or torch.cuda.current_stream(t.device)).cuda_stream)


def avg_pool(fmap: torch.Tensor, s: int, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Second pyramid level: [F, H, W, D] bf16 -> [F, H // s, W // s, D] bf16."""
    F, H, W, D = fmap.shape
    assert fmap.dtype == torch.bfloat16 and fmap.is_contiguous()
    if out is None:
        out = torch.empty((F, H // s, W // s, D), dtype=torch.bfloat16, device=fmap.device)
    r = native.lib().dpc_avg_pool(_p(fmap), F, H, W, D, s, _p(out), _stream(fmap, stream))
    if r != native.BA_OK:
        raise BAError(r, "dpc_avg_pool failed")
    return out


def correlation(level0: torch.Tensor, level1: torch.Tensor, scale1: float, gmap: torch.Tensor,
                coords: torch.Tensor, kk: torch.Tensor, jj: torch.Tensor,
                out: Optional[torch.Tensor] = None, status: Optional[torch.Tensor] = None,
                stream=None) -> torch.Tensor:
    """Eq. 4 at both pyramid levels.  level0 [F, H0, W0, D], level1
    [F, H1, W1, D], gmap [M, p*p, D] bf16; coords [E, p*p, 2] f32 in
    first-level pixels; kk, jj [E] int32.  Returns [E, 2, p*p, 7, 7] f32."""
    for t in (level0, level1, gmap, coords, kk, jj):
        assert t.is_contiguous() and t.device == level0.device
    assert level0.dtype == level1.dtype == gmap.dtype == torch.bfloat16
    assert coords.dtype == torch.float32 and kk.dtype == jj.dtype == torch.int32
    F, H0, W0, D = level0.shape
    _, H1, W1, _ = level1.shape
    M, P2, _ = gmap.shape
    E = coords.shape[0]
    if out is None:
        out = torch.empty((E, 2, P2, 7, 7), dtype=torch.float32, device=level0.device)
    p = DPCProblem()
    p.n_frames, p.channels, p.height0, p.width0, p.height1, p.width1 = F, D, H0, W0, H1, W1
    p.scale1, p.patch_pixels, p.n_patches, p.n_edges = float(scale1), P2, M, E
    p.level0, p.level1, p.gmap, p.coords = _p(level0), _p(level1), _p(gmap), _p(coords)
    p.kk, p.jj, p.out, p.status = _p(kk), _p(jj), _p(out), _p(status)
    r = native.lib().dpc_correlation(ctypes.byref(p), _stream(level0, stream))
    if r != native.BA_OK:
        raise BAError(r, "dpc_correlation failed")
    return out
