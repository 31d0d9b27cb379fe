"""Pins of the soft-aggregation oracle (oracle/agg_oracle.py) to what Eq. 5
fixes independently of its code: a neighbourhood of one edge gives psi(phi(x))
(the gate cancels), a constant gate gives psi of the plain mean of phi, the
result is shared by a neighbourhood and invariant to the order of its edges,
the neighbourhoods are the patch and the (source frame, target frame) pair,
and the group sums equal a library scatter-add."""
import numpy as np
import pytest
import torch

from oracle import agg_oracle as A


def _layers(D, rng, scale=0.3):
    W = [rng.normal(size=(D, D)) * scale for _ in range(3)]
    b = [rng.normal(size=D) * 0.1 for _ in range(3)]
    return W, b


def _graph():
    # 3 frames, 2 patches per frame, every patch joined to every frame
    anchor = np.repeat(np.arange(3), 2)
    kk = np.repeat(np.arange(6), 3)
    jj = np.tile(np.arange(3), 6)
    return anchor, kk, jj


def test_single_edge_neighbourhood_is_psi_of_phi():
    rng = np.random.default_rng(0)
    D = 8
    (Wg, Wv, Wo), (bg, bv, bo) = _layers(D, rng)
    x = rng.normal(size=(3, D))
    kk, jj, anchor = np.array([0, 1, 2]), np.array([0, 0, 0]), np.array([0, 1, 2])
    out = A.soft_aggregate(A.PATCH, x, kk, jj, anchor, 3, Wg, bg, Wv, bv, Wo, bo)
    want = (x @ Wv.T + bv) @ Wo.T + bo
    np.testing.assert_allclose(out, want, rtol=1e-12, atol=1e-12)


def test_constant_gate_gives_plain_mean():
    rng = np.random.default_rng(1)
    D = 6
    (_, Wv, Wo), (_, bv, bo) = _layers(D, rng)
    Wg, bg = np.zeros((D, D)), np.zeros(D)          # sigma = 1/2 everywhere
    anchor, kk, jj = _graph()
    x = rng.normal(size=(len(kk), D))
    out = A.soft_aggregate(A.PATCH, x, kk, jj, anchor, 3, Wg, bg, Wv, bv, Wo, bo)
    for k in range(6):
        sel = kk == k
        want = (x[sel] @ Wv.T + bv).mean(0) @ Wo.T + bo
        np.testing.assert_allclose(out[sel], np.broadcast_to(want, out[sel].shape), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("mode", [A.PATCH, A.FRAME])
def test_neighbourhoods_share_the_result_and_ignore_order(mode):
    rng = np.random.default_rng(2)
    D = 5
    (Wg, Wv, Wo), (bg, bv, bo) = _layers(D, rng)
    anchor, kk, jj = _graph()
    x = rng.normal(size=(len(kk), D))
    out = A.soft_aggregate(mode, x, kk, jj, anchor, 3, Wg, bg, Wv, bv, Wo, bo)
    key = kk if mode == A.PATCH else anchor[kk] * 3 + jj
    for k in np.unique(key):
        sel = np.nonzero(key == k)[0]
        assert np.allclose(out[sel], out[sel[0]], rtol=0, atol=1e-13)
    # the frame neighbourhood of (source frame a, target j) is the edges of
    # frame a's two patches into j
    if mode == A.FRAME:
        assert all((key == a * 3 + j).sum() == 2 for a in range(3) for j in range(3))
    p = rng.permutation(len(kk))
    out_p = A.soft_aggregate(mode, x[p], kk[p], jj[p], anchor, 3, Wg, bg, Wv, bv, Wo, bo)
    np.testing.assert_allclose(out_p, out[p], rtol=1e-12, atol=1e-12)


def test_group_sums_equal_a_library_scatter_add():
    rng = np.random.default_rng(3)
    D = 7
    (Wg, Wv, Wo), (bg, bv, bo) = _layers(D, rng)
    anchor, kk, jj = _graph()
    x = rng.normal(size=(len(kk), D))
    out, it = A.soft_aggregate(A.FRAME, x, kk, jj, anchor, 3, Wg, bg, Wv, bv, Wo, bo, intermediates=True)
    key = torch.as_tensor(anchor[kk] * 3 + jj)
    s = torch.sigmoid(torch.as_tensor(x) @ torch.as_tensor(Wg).T + torch.as_tensor(bg))
    f = torch.as_tensor(x) @ torch.as_tensor(Wv).T + torch.as_tensor(bv)
    num = torch.zeros(9, D, dtype=torch.float64).index_add_(0, key, s * f)
    den = torch.zeros(9, D, dtype=torch.float64).index_add_(0, key, s)
    y = (num / den)[key]
    want = y @ torch.as_tensor(Wo).T + torch.as_tensor(bo)
    np.testing.assert_allclose(out, want.numpy(), rtol=1e-12, atol=1e-12)
    assert np.all(it["n"] == 2)
