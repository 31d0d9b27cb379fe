"""Pins of the correlation oracle (oracle/corr_oracle.py) to what Eq. 4 and
the average-pooled pyramid fix independently of its code: integer grid
points reduce to plain feature lookups, a linear feature field is sampled
exactly, a half-pixel point is the mean of its four neighbours, a shift of
the reprojection by a whole pixel shifts the 7 x 7 grid, points outside the
map see zero features, the result is linear in the patch features, and the
pooled level equals a reshape-and-mean."""
import numpy as np
import pytest

from oracle import corr_oracle as C


def _maps(F=3, H=9, W=11, D=8, seed=0):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(F, H, W, D)), rng.normal(size=(5, 4, D))


def test_integer_points_are_feature_lookups():
    fm, g = _maps()
    coords = np.array([[[4.0, 3.0], [0.0, 0.0], [10.0, 8.0], [2.0, 7.0]]])   # (x, y)
    kk, jj = np.array([2]), np.array([1])
    out = C.correlation([fm], [1], g, coords, kk, jj)[0, 0]
    H, W = fm.shape[1:3]
    for q in range(4):
        x, y = coords[0, q]
        for a in range(7):
            for b in range(7):
                yy, xx = int(y) + a - 3, int(x) + b - 3
                want = float(fm[1, yy, xx] @ g[2, q]) if 0 <= yy < H and 0 <= xx < W else 0.0
                assert out[q, a, b] == pytest.approx(want, abs=1e-12)


def test_linear_field_is_sampled_exactly():
    """f(x, y) = a x + b y + c per channel: a bilinear sample of interior
    points equals the field itself, so C = <g, a (x+dx) + b (y+dy) + c>."""
    H, W, D = 20, 24, 6
    rng = np.random.default_rng(1)
    a, b, c = rng.normal(size=D), rng.normal(size=D), rng.normal(size=D)
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    fm = (xx[..., None] * a + yy[..., None] * b + c)[None]
    g = rng.normal(size=(1, 2, D))
    coords = np.array([[[10.3, 9.75], [12.5, 8.125]]])
    out = C.correlation([fm], [1], g, coords, np.array([0]), np.array([0]))[0, 0]
    for q in range(2):
        x, y = coords[0, q]
        for al in range(7):
            for be in range(7):
                f = a * (x + be - 3) + b * (y + al - 3) + c
                assert out[q, al, be] == pytest.approx(float(f @ g[0, q]), rel=1e-12, abs=1e-12)


def test_half_pixel_is_mean_of_four():
    fm, g = _maps(seed=2)
    coords = np.array([[[5.5, 4.5]]])
    out = C.correlation([fm], [1], g[:, :1], coords, np.array([3]), np.array([2]))[0, 0, 0]
    f = fm[2]
    # grid centre (alpha = beta = 3): the point (5.5, 4.5) itself
    want = 0.25 * (f[4, 5] + f[4, 6] + f[5, 5] + f[5, 6]) @ g[3, 0]
    assert out[3, 3] == pytest.approx(float(want), abs=1e-12)


def test_whole_pixel_shift_shifts_the_grid():
    fm, g = _maps(H=30, W=30, seed=3)
    c0 = np.array([[[12.3, 14.6]]])
    c1 = c0 + np.array([1.0, 0.0])
    c2 = c0 + np.array([0.0, -2.0])
    g = g[:, :1]
    o0 = C.correlation([fm], [1], g, c0, np.array([1]), np.array([0]))[0, 0, 0]
    o1 = C.correlation([fm], [1], g, c1, np.array([1]), np.array([0]))[0, 0, 0]
    o2 = C.correlation([fm], [1], g, c2, np.array([1]), np.array([0]))[0, 0, 0]
    np.testing.assert_allclose(o1[:, :6], o0[:, 1:], rtol=1e-12, atol=1e-12)   # x + 1: beta shifts by one
    np.testing.assert_allclose(o2[2:, :], o0[:5, :], rtol=1e-12, atol=1e-12)   # y - 2: alpha shifts back by two


def test_outside_the_map_is_zero_and_the_edge_is_partial():
    fm, g = _maps(seed=4)
    far = np.array([[[-50.0, 3.0], [3.0, 400.0]]])
    out = C.correlation([fm], [1], g[:, :2], far, np.array([0]), np.array([0]))
    assert np.all(out == 0.0)
    # a point half a pixel left of the first column: its grid centre sees
    # half of column 0 and half of the zero outside
    edge = np.array([[[-0.5, 2.0]]])
    o = C.correlation([fm], [1], g[:, :1], edge, np.array([0]), np.array([0]))[0, 0, 0]
    assert o[3, 3] == pytest.approx(float(0.5 * fm[0, 2, 0] @ g[0, 0]), abs=1e-12)


def test_linear_in_patch_features_and_second_level_scaling():
    fm, g = _maps(seed=5)
    rng = np.random.default_rng(6)
    coords = rng.uniform(-2, 12, size=(4, 4, 2))
    kk, jj = np.array([0, 1, 2, 4]), np.array([0, 2, 1, 1])
    fm1 = rng.normal(size=(3, 5, 6, 8))
    o = C.correlation([fm, fm1], [1, 2], g, coords, kk, jj)
    g2 = rng.normal(size=g.shape)
    o2 = C.correlation([fm, fm1], [1, 2], g2, coords, kk, jj)
    o12 = C.correlation([fm, fm1], [1, 2], g + 3.0 * g2, coords, kk, jj)
    np.testing.assert_allclose(o12, o + 3.0 * o2, rtol=1e-10, atol=1e-10)
    # the second level at coordinates c equals a first-level evaluation on
    # that map at c / 2
    alone = C.correlation([fm1], [1], g, coords / 2.0, kk, jj)
    np.testing.assert_array_equal(o[:, 1], alone[:, 0])


def test_abs_bound_dominates():
    fm, g = _maps(seed=7)
    rng = np.random.default_rng(8)
    coords = rng.uniform(-1, 11, size=(3, 4, 2))
    kk, jj = np.array([0, 3, 4]), np.array([2, 0, 1])
    o = C.correlation([fm], [1], g, coords, kk, jj)
    a = C.correlation_abs([fm], [1], g, coords, kk, jj)
    assert np.all(np.abs(o) <= a + 1e-12)


def test_avg_pool_is_reshape_mean():
    rng = np.random.default_rng(9)
    fm = rng.normal(size=(2, 13, 17, 3))
    for s in (2, 4):
        h, w = 13 // s, 17 // s
        want = fm[:, :h * s, :w * s].reshape(2, h, s, w, s, 3).mean(axis=(2, 4))
        np.testing.assert_allclose(C.avg_pool(fm, s), want, rtol=1e-13, atol=1e-14)
    const = np.full((1, 8, 8, 2), 1.25)
    assert np.all(C.avg_pool(const, 4) == 1.25)
