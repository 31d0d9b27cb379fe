"""Degenerate inputs on the GPU path: depth-only windows, empty graphs,
duplicate edges, unsorted patches, zero weights, zero iterations, a single
frame, too many edges on one patch, an empty batch."""
import numpy as np
import pytest
import torch

from oracle import ba_oracle as O
from paper_2208_04726_amd import synth
from tests.gpu_util import compare, need_gpu, solve_gpu

pytestmark = pytest.mark.gpu

FP64_TOL = (1e-6, 1e-4, 1e-6)


def _check_fp64(w, out):
    pr, dr = O.solve(w)
    dc, drot, dd = compare(out[0], out[1], pr, dr)
    assert dc < FP64_TOL[0] and drot < FP64_TOL[1] and dd < FP64_TOL[2], (dc, drot, dd)


@pytest.mark.parametrize("schedule", ["split", "fused"])
def test_depth_only_window(schedule):
    """Every pose fixed (n = 0): only the inverse depths move (the depth-only
    training stage of Sec. 3.2), per patch, as in the oracle."""
    need_gpu()
    w = synth.make_window(6, 10, 3, seed=[40], outlier_frac=0.1, n_fixed=6)
    (r,), st = solve_gpu([w], "fp64", schedule)
    assert st[0] == 0
    assert np.array_equal(r[0], w.poses)
    _check_fp64(w, r)


def test_unsorted_patches_match_oracle():
    """Patches not grouped by source frame (and edges in random order)."""
    need_gpu()
    w = synth.plain_fp64_window(4)
    rng = np.random.default_rng(3)
    perm = rng.permutation(w.n_patches)          # new patch i = old patch perm[i]
    inv = np.argsort(perm)
    u = w.copy()
    u.patches, u.anchor = w.patches[perm].copy(), w.anchor[perm].copy()
    u.depth_gt = w.depth_gt[perm].copy()
    u.kk = inv[w.kk].astype(np.int32)
    u = synth.shuffled(u, 9)
    (r,), st = solve_gpu([u], "fp64", "split")
    assert st[0] == 0
    _check_fp64(u, r)


def test_duplicate_edges_are_independent_residuals():
    need_gpu()
    w = synth.plain_fp64_window(5)
    d = w.copy()
    pick = np.arange(0, w.n_edges, 7)
    d.kk = np.concatenate([w.kk, w.kk[pick]])
    d.jj = np.concatenate([w.jj, w.jj[pick]])
    d.targets = np.concatenate([w.targets, w.targets[pick] + 0.5])
    d.weights = np.concatenate([w.weights, w.weights[pick] * 0.5])
    for sched in ("split", "fused"):
        (r,), st = solve_gpu([d], "fp64", sched)
        assert st[0] == 0
        _check_fp64(d, r)


def test_zero_weights_leave_state_unchanged():
    need_gpu()
    w = synth.plain_fp64_window(6)
    w.weights = np.zeros_like(w.weights)
    (r,), st = solve_gpu([w], "fp64", "split")
    assert st[0] == 0
    assert np.abs(r[0] - w.poses).max() < 1e-12
    assert np.array_equal(r[1], w.patches[:, 2])


def test_zero_iterations_copy_inputs():
    need_gpu()
    w = synth.method_scale_window(6)
    for sched in ("split", "fused"):
        (r,), st = solve_gpu([w], "fp32", sched, iterations=0)
        assert np.array_equal(r[0], w.poses) and np.array_equal(r[1], w.patches[:, 2])


def test_windows_without_edges_or_patches():
    """A single free frame with only self-edges, a window with no edges and a
    window with no patches sit in one batch with a normal window."""
    need_gpu()
    single = synth.make_window(1, 6, 0, seed=[41], n_fixed=0)        # self-edges only
    noedge = synth.make_window(4, 5, 2, seed=[42])
    noedge.kk = noedge.kk[:0]
    noedge.jj = noedge.jj[:0]
    noedge.targets = noedge.targets[:0]
    noedge.weights = noedge.weights[:0]
    nopatch = synth.make_window(3, 1, 1, seed=[43])
    nopatch.patches = nopatch.patches[:0]
    nopatch.anchor = nopatch.anchor[:0]
    nopatch.kk = nopatch.kk[:0]
    nopatch.jj = nopatch.jj[:0]
    nopatch.targets = nopatch.targets[:0]
    nopatch.weights = nopatch.weights[:0]
    normal = synth.plain_fp64_window(8)
    wins = [single, noedge, normal, nopatch]
    out, st = solve_gpu(wins, "fp64", "split")
    assert (st == 0).all(), st
    for w, r in zip((single, noedge, nopatch), (out[0], out[1], out[3])):
        assert np.abs(r[0] - w.poses).max() < 1e-12
        assert np.array_equal(r[1], w.patches[:, 2])
    _check_fp64(normal, out[2])


def test_patch_degree_above_64_is_reported():
    need_gpu()
    w = synth.plain_fp64_window(9)
    d = w.copy()
    extra = 70
    d.kk = np.concatenate([w.kk, np.full(extra, 3, np.int32)])
    d.jj = np.concatenate([w.jj, np.full(extra, (w.anchor[3] + 1) % w.n_frames, np.int32)])
    d.targets = np.concatenate([w.targets, np.repeat(w.targets[:1], extra, 0)])
    d.weights = np.concatenate([w.weights, np.repeat(w.weights[:1], extra, 0)])
    out, st = solve_gpu([w, d], "fp64", "split")
    assert st[0] == 0 and st[1] & 8
    assert np.array_equal(out[1][0], d.poses) and np.array_equal(out[1][1], d.patches[:, 2])
    _check_fp64(w, out[0])


def test_empty_batch():
    need_gpu()
    from paper_2208_04726_amd.solver import Solver, make_batch
    s = Solver(precision="fp32", max_windows=4, max_patches=16, max_edges=64)
    b = make_batch([], "fp32")
    po, do = s.solve(b)
    torch.cuda.synchronize()
    assert po.shape == (0, 7) and do.shape == (0,)
    assert len(s.status()) == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_irregular_graph_method_scale(precision):
    """Each patch of a 22x96 window keeps a random 85% of its edges, so the
    patches of a source frame have different target sequences: the general
    pair-table path (LDS tables per lane segment), against the oracle."""
    need_gpu()
    w = synth.method_scale_window(6)
    rng = np.random.default_rng(61)
    keep = rng.uniform(size=w.n_edges) < 0.85
    d = w.copy()
    d.kk, d.jj = w.kk[keep].copy(), w.jj[keep].copy()
    d.targets, d.weights = w.targets[keep].copy(), w.weights[keep].copy()
    (r,), st = solve_gpu([d], precision, "split")
    assert st[0] == 0
    pr, dr = O.solve(d)
    dc, drot, dd = compare(r[0], r[1], pr, dr)
    print(precision, "irregular 22x96:", f"{dc:.2e} m {drot:.2e} deg depth {dd:.2e}")
    tol = FP64_TOL if precision == "fp64" else (1e-4, 1e-2, 1e-3)
    assert dc < tol[0] and drot < tol[1] and dd < tol[2], (dc, drot, dd)


@pytest.mark.parametrize("shape,precision", [((22, 96, 13), "fp64"), ((22, 96, 13), "fp32"),
                                             ((64, 256, 16), "fp32")])
def test_interleaved_patches_equal_frame_ordered_input(shape, precision):
    """Patches of different source frames interleaved at random, each frame's
    patches keeping their relative order, edges left in their input order
    (so neither patches nor edges are grouped any more).  The preparation
    orders positions by (source frame, patch index) and each patch's edges by
    (target frame, input index), which is the order of the frame-ordered
    input: the solve must be bitwise the same.  Exercises the stable ordering
    of unsorted patches at up to 256 patches per frame and the gathered edge
    layout."""
    need_gpu()
    F, ppf, r = shape
    w = synth.make_window(F, ppf, r, seed=[41, F], outlier_frac=0.1, fp32=True)
    rng = np.random.default_rng(5)
    labels = rng.permutation(np.asarray(w.anchor))
    by_frame = [list(np.nonzero(np.asarray(w.anchor) == a)[0]) for a in range(F)]
    nxt = np.zeros(F, np.int64)
    order = np.empty(w.n_patches, np.int64)          # new patch i = old patch order[i]
    for i, a in enumerate(labels):
        order[i] = by_frame[a][nxt[a]]
        nxt[a] += 1
    inv = np.argsort(order)
    u = w.copy()
    u.patches, u.anchor = w.patches[order].copy(), w.anchor[order].copy()
    u.depth_gt = w.depth_gt[order].copy()
    u.kk = inv[w.kk].astype(np.int32)
    assert np.any(np.diff(u.anchor) < 0) and np.any(np.diff(u.kk) < 0)
    (a_,), sa = solve_gpu([w], precision, "split")
    (b_,), sb = solve_gpu([u], precision, "split")
    assert sa[0] == 0 and sb[0] == 0
    assert np.array_equal(a_[0], b_[0])
    assert np.array_equal(a_[1][order], b_[1])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_depth_only_method_scale(precision):
    """Structure-only BA at method scale: 22 x 96, r = 13, every pose fixed
    (the depth-only training stage, Sec. 3.2).  Poses come back bitwise
    unchanged; inverse depths match the oracle, FP64 within 1e-6 relative,
    FP32 by the FP32 depth criterion (tests/rounding.py)."""
    need_gpu()
    from tests.rounding import check_depths, depth_sensitivity
    w = synth.make_window(22, 96, 13, seed=[42], outlier_frac=0.1, fp32=True, n_fixed=22)
    (r,), st = solve_gpu([w], precision, "split")
    assert st[0] == 0
    assert np.array_equal(r[0], w.poses)
    pr, dr = O.solve(w)
    if precision == "fp64":
        _check_fp64(w, r)
    else:
        check_depths(r[1], dr, depth_sensitivity(w), label="depth-only 22x96")
