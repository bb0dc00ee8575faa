"""Pins of the data-cost oracle (Sec. 2 eq. Cost_value, Sec. 5.1 eq. Cost_cmp), no GPU."""
import numpy as np

import synth
from oracle import dsi_ref as D


def test_hand_example():
    """3 x 2 images; stereo labels d = 0, 1 compare I0(x, y) with I1(x - d, y)."""
    i0 = np.array([[10, 20, 30], [0, 5, 9]], np.uint8)
    i1 = np.array([[12, 14, 40], [3, 0, 20]], np.uint8)
    c = D.dsi(i0, i1, 2, 1, 0, 0, -1, 1, 1, 100)
    # d = 0: |12-10| |14-20| |40-30| / |3-0| |0-5| |20-9|
    assert c[..., 0].tolist() == [[2, 6, 10], [3, 5, 11]]
    # d = 1: x = 0 leaves the image; |12-20| |14-30| / |3-5| |0-9|
    assert c[..., 1].tolist() == [[100, 8, 16], [100, 2, 9]]
    c2 = D.dsi(i0, i1, 2, 1, 0, 0, -1, 1, 2, 50)
    assert c2[..., 0].tolist() == [[4, 36, 50], [9, 25, 50]]
    assert c2[..., 1].tolist() == [[50, 50, 50], [50, 4, 50]]


def test_composite_by_hand():
    """Three views, labels d = 0, 1: min of I1 at x - d and I2 at x + d (eq. Cost_cmp with v = -d)."""
    i0 = np.array([[10, 20, 30]], np.uint8)
    i1 = np.array([[11, 25, 0]], np.uint8)
    i2 = np.array([[40, 19, 33]], np.uint8)
    c = D.dsi(i0, i1, 2, 1, 0, 0, -1, 1, 1, 100, i2=i2)
    # d = 0: min(|11-10|, |40-10|), min(|25-20|, |19-20|), min(|0-30|, |33-30|)
    assert c[..., 0].tolist() == [[1, 1, 3]]
    # d = 1: view 1 at x - 1 (outside at x = 0), view 2 at x + 1 (outside at x = 2):
    # min(100, |19-10|), min(|11-20|, |33-20|), min(|25-30|, 100)
    assert c[..., 1].tolist() == [[9, 9, 5]]


def test_matches_the_synthetic_stereo_generator():
    """The stereo workloads' cost (written separately in synth) is eq. Cost_value with l2 = 1."""
    p = synth.stereo_problem(seed=3, W=96, H=40, Q=12)
    left, right = p.meta["frames"]
    assert np.array_equal(D.dsi(left, right, 12, 1, 0, 0, -1, 1, 1, 50), p.cost.astype(np.int64))


def test_matches_the_synthetic_motion_generator():
    i0, i1, _, _ = synth.motion_frames(seed=4, W=48, H=36, r=3)
    ref = synth.motion_cost(i0, i1, 3, 2500)
    assert np.array_equal(D.dsi(i0, i1, 7, 7, -3, -3, 1, 1, 2, 2500), ref)


def test_composite_with_the_same_second_view_is_symmetric():
    """With I2 = I1 and a label range symmetric about 0, C_cmp(v) = min(C(v), C(-v)): the single-view
    volume and its label-reversed copy."""
    rng = np.random.default_rng(9)
    i0 = rng.integers(0, 256, (20, 26), dtype=np.uint8)
    i1 = rng.integers(0, 256, (20, 26), dtype=np.uint8)
    one = D.dsi(i0, i1, 5, 3, -2, -1, 1, 1, 2, 3000)
    both = D.dsi(i0, i1, 5, 3, -2, -1, 1, 1, 2, 3000, i2=i1)
    assert np.array_equal(both, np.minimum(one, one[..., ::-1]))
    assert (both <= one).all()
