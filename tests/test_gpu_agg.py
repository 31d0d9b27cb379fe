"""Parity of the gfx950 soft aggregation (dpa_softagg, through the C ABI)
with the FP64 oracle.

Bound, by first-order propagation of FP32 rounding through each stage (u =
2^-24, gamma_n = n u / (1 - n u)), from the oracle's own intermediates:
  z, f (gate and value layers, D exact bf16 products summed in FP32, plus the
  bias): within gamma_(D+1) (|x| |W|^T + |b|);
  sigma: within z's error / 4 (the sigmoid's slope) + 6 u sigma (exp, add,
  divide);
  sigma*phi: from both, + u |sigma*phi|;
  the neighbourhood sums of n terms in FP32: the terms' errors + gamma_n of
  the summed magnitudes;
  y = A / B: (e_A + |y| e_B) / (B - e_B) + u |y|;
  psi: |W_out| e_y + gamma_(2D+1) (|W_out| |y| + |b_out|)."""
import numpy as np
import pytest
import torch

from oracle import agg_oracle as A
from paper_2208_04726_amd import synth
from tests.gpu_util import need_gpu

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def gamma(n):
    return n * U / (1 - n * U)


def _dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype).contiguous()


def run_gpu(wl, mode, kk=None, jj=None, status=None):
    from paper_2208_04726_amd import agg
    out = agg.softagg(mode, _dev(wl.x, torch.bfloat16), _dev(wl.kk if kk is None else kk, torch.int32),
                      _dev(wl.jj if jj is None else jj, torch.int32), _dev(wl.anchor, torch.int32), wl.n_frames,
                      [_dev(w, torch.bfloat16) for w in wl.w], [_dev(b, torch.float32) for b in wl.b],
                      status=status)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def bound(wl, mode, it):
    x = np.abs(wl.x.astype(np.float64))
    Wg, Wv, Wo = [np.abs(w.astype(np.float64)) for w in wl.w]
    bg, bv, bo = [np.abs(b.astype(np.float64)) for b in wl.b]
    D = x.shape[1]
    ez = gamma(D + 1) * (x @ Wg.T + bg)
    ef = gamma(D + 1) * (x @ Wv.T + bv)
    s, f = it["s"], it["f"]
    es = 0.25 * ez + 6 * U * s
    p = s * f
    ep = s * ef + np.abs(f) * es + es * ef + U * np.abs(p)
    G = len(it["n"])
    g = it["group"]
    eA = np.zeros((G, D))
    eB = np.zeros((G, D))
    mA = np.zeros((G, D))
    mB = np.zeros((G, D))
    np.add.at(eA, g, ep)
    np.add.at(eB, g, es)
    np.add.at(mA, g, np.abs(p))
    np.add.at(mB, g, s)
    n = it["n"][:, None]
    eA += gamma(n) * mA
    eB += gamma(n) * mB
    y, B = it["y"], it["B"]
    ey = (eA + np.abs(y) * eB) / (B - eB) + U * np.abs(y)
    eo = ey @ Wo.T + gamma(2 * D + 1) * (np.abs(y) @ Wo.T + bo)
    return eo[g]


def check(wl, mode, got, edges=None):
    ref, it = A.soft_aggregate(mode, wl.x, wl.kk, wl.jj, wl.anchor, wl.n_frames, wl.w[0], wl.b[0], wl.w[1],
                               wl.b[1], wl.w[2], wl.b[2], intermediates=True)
    bd = bound(wl, mode, it)
    sel = slice(None) if edges is None else edges
    err = np.abs(got[sel] - ref[sel])
    worst = float((err / bd[sel]).max())
    print(f"  mode {mode}: {err.shape[0]} edges, max |err| {err.max():.2e}, worst err / bound {worst:.3f}, "
          f"neighbourhoods {len(it['n'])} (largest {it['n'].max()})")
    assert np.all(err <= bd[sel])


@pytest.mark.parametrize("dim", [128, 256, 384, 512])
@pytest.mark.parametrize("mode", [A.PATCH, A.FRAME])
def test_small_graph_matches_oracle(mode, dim):
    need_gpu()
    wl = synth.aggregation_workload(6, 8, 3, seed=[2208, 11, dim], dim=dim)
    check(wl, mode, run_gpu(wl, mode))


@pytest.mark.parametrize("mode", [A.PATCH, A.FRAME])
def test_method_scale_graph_matches_oracle(mode):
    """The 22 x 96, radius-13 graph (39,552 edges, 384 channels): every edge;
    frame neighbourhoods of 96 edges span several 64-row chunks."""
    need_gpu()
    wl = synth.method_scale_aggregation(0)
    got = run_gpu(wl, mode)
    check(wl, mode, got)
    again = run_gpu(wl, mode)
    assert np.array_equal(got, again)      # fixed summation order: bitwise repeatable


def test_graph_reuse_with_new_hidden_states():
    """graph_ready: a second call on new hidden states reuses the
    neighbourhoods the first call left in the workspace."""
    need_gpu()
    from paper_2208_04726_amd import agg
    wl = synth.aggregation_workload(8, 12, 4, seed=[2208, 13], dim=256)
    wl2 = synth.aggregation_workload(8, 12, 4, seed=[2208, 14], dim=256)   # same graph, new states and layers
    assert np.array_equal(wl.kk, wl2.kk) and np.array_equal(wl.jj, wl2.jj)
    kk, jj, anc = _dev(wl.kk, torch.int32), _dev(wl.jj, torch.int32), _dev(wl.anchor, torch.int32)
    ws = torch.empty((agg.workspace_bytes(A.FRAME, 256, wl.n_edges, len(wl.anchor), wl.n_frames),),
                     dtype=torch.uint8, device="cuda")
    outs = []
    for w, ready in ((wl, False), (wl2, True)):
        o = agg.softagg(A.FRAME, _dev(w.x, torch.bfloat16), kk, jj, anc, w.n_frames,
                        [_dev(m, torch.bfloat16) for m in w.w], [_dev(b, torch.float32) for b in w.b],
                        workspace=ws, graph_ready=ready)
        torch.cuda.synchronize()
        outs.append(o.cpu().numpy().astype(np.float64))
    check(wl, A.FRAME, outs[0])
    check(wl2, A.FRAME, outs[1])


def test_bad_indices_give_zero_rows_and_a_status_bit():
    need_gpu()
    wl = synth.aggregation_workload(5, 6, 2, seed=[2208, 12], dim=128)
    kk, jj = wl.kk.copy(), wl.jj.copy()
    kk[3] = -1
    jj[7] = 99
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    got = run_gpu(wl, A.FRAME, kk=kk, jj=jj, status=status)
    assert np.all(got[3] == 0.0) and np.all(got[7] == 0.0) and int(status.item()) & 4
    keep = np.setdiff1d(np.arange(len(kk)), [3, 7])
    wl2 = synth.AggWorkload(x=wl.x[keep], kk=kk[keep], jj=jj[keep], anchor=wl.anchor, n_frames=wl.n_frames,
                            w=wl.w, b=wl.b)
    check(wl2, A.FRAME, got[keep])
