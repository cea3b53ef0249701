"""Pins of the RSSI head's oracle (paper Sec. 7.2: global average pooling of the
spectrum map) by properties the definition fixes, independent of its code."""
import numpy as np
import pytest

from oracle import model as M
from oracle import rssi as R


def _scene(H, W, rows):
    """Gaussians from rows (mx, my, lsx, lsy, rot, logit, amp, depth)."""
    a = np.asarray(rows, np.float64)
    g = {k: np.ascontiguousarray(a[:, j], np.float32) for j, k in enumerate(
        ("mean_x", "mean_y", "log_scale_x", "log_scale_y", "rotation", "opacity_logit", "amplitude", "depth"))}
    return M.Scene.from_arrays(g, H, W)


def test_one_pixel_grid_is_the_pixel():
    # a single Gaussian centred on the only pixel: A = amp * min(0.99, sigmoid(logit)); rssi is that value
    s = _scene(1, 1, [[0.0, 0.0, 0.5, 0.3, 0.2, 0.4, 0.75, 1.0]])
    r, res = R.rssi_query(s, None, None)
    o = 1.0 / (1.0 + np.exp(-np.float64(np.float32(0.4))))
    assert r == pytest.approx(np.float64(np.float32(0.75)) * min(o, np.float64(np.float32(0.99))), rel=1e-14)


def test_disjoint_gaussians_add():
    # two Gaussians whose 3-sigma boxes share no pixel: the pooled value of both is the sum of each alone
    H, W = 16, 48
    a = [8.0, 8.0, 0.0, 0.2, 0.3, 0.5, 0.8, 1.0]
    b = [36.0, 7.0, 0.3, 0.0, 1.1, -0.2, 0.6, 2.0]
    r_ab, _ = R.rssi_query(_scene(H, W, [a, b]), None, None)
    r_a, _ = R.rssi_query(_scene(H, W, [a]), None, None)
    r_b, _ = R.rssi_query(_scene(H, W, [b]), None, None)
    assert r_ab == pytest.approx(r_a + r_b, rel=1e-13)


def test_whole_pixel_shift_inside_grid_keeps_value():
    H, W = 32, 32
    g0 = [10.0, 12.0, 0.4, 0.1, 0.7, 0.9, 0.9, 1.0]
    g1 = [17.0, 19.0] + g0[2:]
    r0, res0 = R.rssi_query(_scene(H, W, [g0]), None, None)
    r1, _ = R.rssi_query(_scene(H, W, [g1]), None, None)
    assert r0 > 0 and r1 == pytest.approx(r0, rel=1e-13)
    # and the value is the plain mean of the spectrum over H x W pixels (not over the nonzero ones)
    assert r0 == pytest.approx(res0.C.sum() / (H * W), rel=1e-14)
    assert np.count_nonzero(res0.C) < H * W


def test_empty_scene_is_zero():
    s = _scene(16, 16, [[-100.0, -100.0, 0.0, 0.0, 0.0, 0.0, 1.0, 1.0]])
    r, _ = R.rssi_query(s, None, None)
    assert r == 0.0


def test_pixel_weights_sum_to_the_gradient():
    w = R.pixel_weights(3.0, 16, 16)
    assert w.shape == (256,) and w.sum() == pytest.approx(3.0, rel=1e-15)
