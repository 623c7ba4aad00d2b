"""Pins of the oracle's edge front end (Sobel gradient, ALPHA/BETA sets of
Sec. 3) against values fixed independently of it: a hand-computed patch,
step and diagonal edges whose class is geometric, scipy's Sobel filter on
random images, and the transpose symmetry."""
import numpy as np
import pytest

import oracle


def test_hand_computed_patch():
    g = np.zeros((5, 5), np.uint8)
    g[1:4, 1:4] = np.arange(1, 10).reshape(3, 3)
    # centre (2, 2): Gx = (3 + 2*6 + 9) - (1 + 2*4 + 7) = 8,
    #                Gy = (7 + 2*8 + 9) - (1 + 2*2 + 3) = 24, |G|^2 = 640
    x, y, beta = oracle.sobel_partition(g, 25)   # 625 < 640
    assert (2, 2) in set(zip(x.tolist(), y.tolist()))
    k = list(zip(x.tolist(), y.tolist())).index((2, 2))
    assert not beta[k]                            # |Gx| <= |Gy|: ALPHA
    x, y, _ = oracle.sobel_partition(g, 26)      # 676 > 640
    assert (2, 2) not in set(zip(x.tolist(), y.tolist()))


def test_steps_and_diagonal_classes():
    v = np.zeros((8, 9), np.uint8)
    v[:, 5:] = 200                                # vertical edge: a steep image line
    x, y, beta = oracle.sobel_partition(v, 10)
    assert len(x) > 0 and beta.all()
    h = np.zeros((9, 8), np.uint8)
    h[5:, :] = 200                                # horizontal edge: a flat image line
    x, y, beta = oracle.sobel_partition(h, 10)
    assert len(x) > 0 and not beta.any()
    d = np.fromfunction(lambda yy, xx: (xx + yy >= 8) * 200, (9, 9)).astype(np.uint8)
    x, y, beta = oracle.sobel_partition(d, 10)   # 45 degrees: |Gx| == |Gy|, slope 1 is in ALPHA
    inner = (x > 1) & (x < 7) & (y > 1) & (y < 7)
    assert inner.any() and not beta[inner].any()


def test_flat_image_and_borders():
    x, y, _ = oracle.sobel_partition(np.full((7, 7), 99, np.uint8), 0)
    assert len(x) == 0
    rng = np.random.default_rng(3)
    g = rng.integers(0, 256, (20, 17)).astype(np.uint8)
    x, y, _ = oracle.sobel_partition(g, 0)
    assert x.min() >= 1 and y.min() >= 1 and x.max() <= 15 and y.max() <= 18
    for shape in ((1, 5), (2, 2), (5, 2)):
        assert len(oracle.sobel_partition(np.ones(shape, np.uint8), 0)[0]) == 0


@pytest.mark.parametrize("seed", range(4))
def test_matches_scipy_sobel(seed):
    ndimage = pytest.importorskip("scipy.ndimage")
    rng = np.random.default_rng(seed)
    g = rng.integers(0, 256, (31, 40)).astype(np.uint8)
    t = 300
    gx = ndimage.sobel(g.astype(np.int64), axis=1)
    gy = ndimage.sobel(g.astype(np.int64), axis=0)
    inner = np.zeros(g.shape, bool)
    inner[1:-1, 1:-1] = True
    want = inner & (gx * gx + gy * gy > t * t)
    yy, xx = np.nonzero(want)
    x, y, beta = oracle.sobel_partition(g, t)
    np.testing.assert_array_equal(x, xx)
    np.testing.assert_array_equal(y, yy)
    np.testing.assert_array_equal(beta, np.abs(gx[yy, xx]) > np.abs(gy[yy, xx]))


def test_transpose_swaps_classes():
    rng = np.random.default_rng(8)
    g = rng.integers(0, 256, (23, 19)).astype(np.uint8)
    x, y, beta = oracle.sobel_partition(g, 200)
    xt, yt, bt = oracle.sobel_partition(g.T.copy(), 200)
    a = {(int(i), int(j)): bool(b) for i, j, b in zip(x, y, beta)}
    b_ = {(int(j), int(i)): bool(b) for i, j, b in zip(xt, yt, bt)}
    assert a.keys() == b_.keys()
    # |Gx| and |Gy| trade places under the transpose; ties stay in ALPHA
    for k in a:
        assert not (a[k] and b_[k])
