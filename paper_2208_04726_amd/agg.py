"""Python front end of the gfx950 soft aggregation (include/dpagg.h):
argument marshalling only, every step runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import native
from .native import BAError, DPAProblem

PATCH, FRAME = 0, 1


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def workspace_bytes(mode: int, dim: int, n_edges: int, n_patches: int, n_frames: int) -> int:
    return int(native.lib().dpa_workspace_bytes(mode, dim, n_edges, n_patches, n_frames))


def softagg(mode: int, x: torch.Tensor, kk: torch.Tensor, jj: torch.Tensor, anchor: torch.Tensor,
            n_frames: int, w: Sequence[torch.Tensor], b: Sequence[torch.Tensor],
            out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
            status: Optional[torch.Tensor] = None, graph_ready: bool = False, stream=None) -> torch.Tensor:
    """Eq. 5 for every edge.  x [E, dim] bf16; kk, jj [E], anchor [M] int32;
    w = (gate, value, output) [dim, dim] bf16 (out, in); b = their [dim] f32
    biases.  graph_ready: reuse the neighbourhoods an earlier call left in
    `workspace` for the same graph.  Returns [E, dim] f32."""
    E, D = x.shape
    M = anchor.shape[0]
    assert x.dtype == torch.bfloat16 and all(t.dtype == torch.bfloat16 for t in w)
    assert all(t.dtype == torch.float32 for t in b) and kk.dtype == jj.dtype == anchor.dtype == torch.int32
    for t in (x, kk, jj, anchor, *w, *b):
        assert t.is_contiguous() and t.device == x.device
    if out is None:
        out = torch.empty((E, D), dtype=torch.float32, device=x.device)
    nb = workspace_bytes(mode, D, E, M, n_frames)
    if nb < 0:
        raise BAError(native.BA_E_INVAL, "bad soft-aggregation sizes")
    if workspace is None:
        workspace = torch.empty((max(nb, 1),), dtype=torch.uint8, device=x.device)
    p = DPAProblem()
    p.mode, p.dim, p.n_edges, p.n_patches, p.n_frames = mode, D, E, M, n_frames
    p.graph_ready = 1 if graph_ready else 0
    p.x, p.kk, p.jj, p.anchor = _p(x), _p(kk), _p(jj), _p(anchor)
    p.w_gate, p.w_val, p.w_out = _p(w[0]), _p(w[1]), _p(w[2])
    p.b_gate, p.b_val, p.b_out = _p(b[0]), _p(b[1]), _p(b[2])
    p.out, p.workspace, p.workspace_bytes, p.status = _p(out), _p(workspace), workspace.numel(), _p(status)
    s = ctypes.c_void_p((stream or torch.cuda.current_stream(x.device)).cuda_stream)
    r = native.lib().dpa_softagg(ctypes.byref(p), s)
    if r != native.BA_OK:
        raise BAError(r, "dpa_softagg failed")
    return out
