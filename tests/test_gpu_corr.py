"""Parity of the gfx950 correlation features (dpc_correlation, dpc_avg_pool,
through the C ABI) with the FP64 correlation oracle.

Bound: the kernel multiplies bfloat16 values exactly in FP32, sums the D
products and combines four lattice products with FP32 bilinear weights, so
by the deterministic summation bound every output is within
gamma_(D+4) = (D+4) u / (1 - (D+4) u), u = 2^-24, of the same sum of
absolute values (oracle.correlation_abs)."""
import numpy as np
import pytest
import torch

from oracle import corr_oracle as C
from paper_2208_04726_amd import synth
from tests.gpu_util import need_gpu

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def gamma(n):
    return n * U32 / (1 - n * U32)


def _dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype).contiguous()


def run_gpu(wl: synth.CorrWorkload, coords=None, kk=None, jj=None, status=None):
    from paper_2208_04726_amd import corr
    c = wl.coords if coords is None else coords
    out = corr.correlation(_dev(wl.fmap0, torch.bfloat16), _dev(wl.fmap1, torch.bfloat16), wl.scale1,
                           _dev(wl.gmap, torch.bfloat16), _dev(c, torch.float32),
                           _dev(wl.kk if kk is None else kk, torch.int32),
                           _dev(wl.jj if jj is None else jj, torch.int32), status=status)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def check(wl, got, edges=None, coords=None):
    c = wl.coords if coords is None else coords
    sel = np.arange(len(wl.kk)) if edges is None else edges
    args = ([wl.fmap0, wl.fmap1], [1, wl.scale1], wl.gmap, c[sel], wl.kk[sel], wl.jj[sel])
    ref = C.correlation(*args)
    mag = C.correlation_abs(*args)
    D = wl.fmap0.shape[-1]
    err = np.abs(got[sel] - ref)
    bound = gamma(D + 4) * mag
    worst = float((err / np.maximum(bound, 1e-300)).max())
    print(f"  {len(sel)} edges: max |err| {err.max():.2e}, worst err / bound {worst:.3f}, "
          f"max |C| {np.abs(ref).max():.1f}")
    assert np.all(err <= bound + 1e-30)


def test_mfma_bf16_lane_layout():
    need_gpu()
    from paper_2208_04726_amd import native
    rng = np.random.default_rng(0)
    A = synth.bf16_exact(rng.normal(size=(16, 32)).astype(np.float32))
    B = synth.bf16_exact(rng.normal(size=(32, 16)).astype(np.float32))
    Ad, Bd = _dev(synth.bf16_bits(A).view(np.int16), torch.int16), _dev(synth.bf16_bits(B).view(np.int16), torch.int16)
    Dd = torch.zeros((16, 16), dtype=torch.float32, device="cuda")
    assert native.lib().dpc_debug_mfma_bf16(Ad.data_ptr(), Bd.data_ptr(), Dd.data_ptr(), None) == 0
    torch.cuda.synchronize()
    ref = A.astype(np.float64) @ B.astype(np.float64)
    bound = gamma(32) * (np.abs(A).astype(np.float64) @ np.abs(B).astype(np.float64))
    assert np.all(np.abs(Dd.cpu().numpy() - ref) <= bound)


@pytest.mark.parametrize("dim,p", [(128, 3), (64, 2), (256, 1), (128, 4)])
def test_small_graph_matches_oracle(dim, p):
    """6 frames x 8 patches, radius 3, 40 x 30 first-level maps: every edge."""
    need_gpu()
    wl = synth.correlation_workload(6, 8, 3, seed=[2208, 6, dim, p], p=p, dim=dim, feature_hw=(30, 40))
    print(f"D={dim} p={p}")
    check(wl, run_gpu(wl))


def test_edge_cases_of_the_sampling():
    """Integer points, the last pixel, half-pixels, points partly and wholly
    outside the map, pixels spread wider than one lattice box (each pixel
    then takes its own 8x8 lattice), and both levels' boundaries."""
    need_gpu()
    wl = synth.correlation_workload(4, 4, 2, seed=[2208, 7], feature_hw=(30, 40), scale1=2)
    E = len(wl.kk)
    c = wl.coords.copy()
    W, H = 40, 30
    cases = [
        [(3.0 + i % 3, 4.0 + i // 3) for i in range(9)],                  # integer points
        [(W - 1.0, H - 1.0)] * 9,                                          # the last pixel
        [(-0.5, 2.5)] * 9,                                                 # half a pixel outside
        [(-5.9, -5.9)] * 9,                                                # lattice corner just inside
        [(-6.5, 10.0)] * 9,                                                # wholly outside
        [(1.0 + 4.3 * i, 2.0 + 3.1 * i) for i in range(9)],                # spread: per-pixel lattices
        [(W + 4.5, H + 4.5)] * 9,                                          # far corner, partly inside
        [(0.25 * i, 29.75 - 0.5 * i) for i in range(9)],                   # second-level border (scale 2)
    ]
    for q, case in enumerate(cases):
        c[q % E] = np.asarray(case, np.float32)
    got = run_gpu(wl, coords=c)
    check(wl, got, coords=c)


def test_nonfinite_coordinates_and_bad_indices():
    need_gpu()
    wl = synth.correlation_workload(4, 4, 2, seed=[2208, 8], feature_hw=(30, 40))
    c = wl.coords.copy()
    c[0, 4] = (np.nan, 3.0)
    c[1, :, 0] = np.inf
    kk, jj = wl.kk.copy(), wl.jj.copy()
    kk[2] = 10_000
    jj[3] = -1
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    got = run_gpu(wl, coords=c, kk=kk, jj=jj, status=status)
    assert np.all(got[0, :, 4] == 0.0) and np.all(got[1] == 0.0)
    assert np.all(got[2] == 0.0) and np.all(got[3] == 0.0)
    assert int(status.item()) & 4
    rest = np.arange(4, len(kk))
    check(wl, got, edges=rest, coords=c)
    # the other pixels of edge 0 are unaffected
    ok = [q for q in range(9) if q != 4]
    ref = C.correlation([wl.fmap0, wl.fmap1], [1, wl.scale1], wl.gmap, c[:1], wl.kk[:1], wl.jj[:1])
    assert np.allclose(got[0][:, ok], ref[0][:, ok], rtol=1e-4, atol=1e-3)


def test_method_scale_graph_sampled_edges():
    """The 22 x 96, radius-13 graph (39,552 edges) over 160 x 120 / 40 x 30
    maps of 128 channels, in the launch the benchmark times; 300 sampled
    edges against the oracle, and the count of edges whose pixels leave the
    map."""
    need_gpu()
    wl = synth.method_scale_correlation(0)
    got = run_gpu(wl)
    rng = np.random.default_rng(1)
    sel = np.sort(rng.choice(wl.n_edges, 300, replace=False))
    check(wl, got, edges=sel)
    assert np.all(np.isfinite(got))


@pytest.mark.parametrize("s", [4, 2, 3])
def test_avg_pool_matches_oracle(s):
    """Pooled level against the oracle's mean: FP32 sum of s*s bfloat16 values
    (within gamma_(s*s) of the summed magnitudes) rounded to the nearest
    bfloat16 (within 2^-8 relative)."""
    need_gpu()
    from paper_2208_04726_amd import corr
    rng = np.random.default_rng(s)
    fm = synth.bf16_exact(rng.normal(size=(3, 30, 41, 128)).astype(np.float32))
    out = corr.avg_pool(_dev(fm, torch.bfloat16), s)
    torch.cuda.synchronize()
    got = out.float().cpu().numpy().astype(np.float64)
    ref = C.avg_pool(fm, s)
    mag = C.avg_pool(np.abs(fm), s)
    d = gamma(s * s + 1) * mag
    bound = 2.0 ** -8 * (np.abs(ref) + d) + d
    print(f"s={s}: max |err| {np.abs(got - ref).max():.2e}")
    assert got.shape == ref.shape
    assert np.all(np.abs(got - ref) <= bound)
