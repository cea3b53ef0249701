"""Pins of the SSIM / hybrid-loss oracle (paper Sec. 4.4, hybrid-loss equation;
SSIM parameters as read in oracle/ssim.py) by closed forms and central
differences, independent of its code."""
import numpy as np
import pytest

from oracle import ssim as S


def test_window_is_a_normalised_symmetric_gaussian():
    w = S.window()
    assert w.shape == (11, 11) and w.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_allclose(w, w.T, rtol=0, atol=0)
    np.testing.assert_allclose(w, w[::-1, ::-1], rtol=0, atol=0)
    # ratio of neighbouring weights along an axis: exp(-((r+1)^2 - r^2) / (2 * 1.5^2))
    assert w[5, 6] / w[5, 5] == pytest.approx(np.exp(-1.0 / 4.5), rel=1e-14)
    assert w[5, 9] / w[5, 5] == pytest.approx(np.exp(-16.0 / 4.5), rel=1e-14)


def test_identical_images_give_one():
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, (20, 33))
    np.testing.assert_allclose(S.ssim_map(x, x), 1.0, rtol=0, atol=1e-14)
    s, g = S.ssim_and_grad(x, x)
    assert s == pytest.approx(1.0, abs=1e-14)
    # SSIM(x, x) is the maximum: the gradient vanishes there
    np.testing.assert_allclose(g, 0.0, atol=1e-12)


def test_symmetric_in_its_arguments():
    rng = np.random.default_rng(1)
    x, y = rng.uniform(0, 1, (2, 17, 24))
    np.testing.assert_allclose(S.ssim_map(x, y), S.ssim_map(y, x), rtol=1e-14, atol=0)


def test_constant_images_in_the_interior():
    # x = a, y = b everywhere: at least 5 pixels from every border the windows see no padding, the variances and
    # the covariance vanish, and S = (2 a b + C1) / (a^2 + b^2 + C1)
    a, b = 0.3, 0.75
    m = S.ssim_map(np.full((15, 16), a), np.full((15, 16), b))
    want = (2 * a * b + S.C1) / (a * a + b * b + S.C1)
    # (the variances are differences E[x^2] - mu^2 of equal values: FP64 rounding of ~1e-16 over C2 = 9e-4)
    np.testing.assert_allclose(m[5:10, 5:11], want, rtol=1e-11)


def test_one_pixel_image_closed_form():
    # a 1 x 1 image sees only the centre weight c of the window (zero padding elsewhere):
    # mu = c x, E[x^2] = c x^2, so sigma_x^2 = (c - c^2) x^2 and sigma_xy = (c - c^2) x y
    x, y = 0.8, 0.35
    g1 = np.exp(-(np.arange(11) - 5.0) ** 2 / 4.5)
    c = (1.0 / g1.sum()) ** 2
    k = c - c * c
    want = ((2 * c * c * x * y + S.C1) * (2 * k * x * y + S.C2)) / \
        ((c * c * (x * x + y * y) + S.C1) * (k * (x * x + y * y) + S.C2))
    assert S.ssim_map(np.array([[x]]), np.array([[y]]))[0, 0] == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("shape", [(12, 14), (7, 30)])
def test_gradient_matches_central_differences(shape):
    rng = np.random.default_rng(shape[1])
    x, y = rng.uniform(0, 1, (2,) + shape)
    s0, g = S.ssim_and_grad(x, y)
    eps = 1e-6
    idx = [tuple(rng.integers(0, n) for n in shape) for _ in range(12)] + [(0, 0), (shape[0] - 1, shape[1] - 1)]
    for ij in idx:
        xp, xm = x.copy(), x.copy()
        xp[ij] += eps
        xm[ij] -= eps
        fd = (S.ssim_and_grad(xp, y)[0] - S.ssim_and_grad(xm, y)[0]) / (2 * eps)
        assert g[ij] == pytest.approx(fd, rel=1e-6, abs=1e-11), ij


def test_hybrid_loss_weights_and_gradient():
    rng = np.random.default_rng(3)
    p, t = rng.uniform(0, 1, (2, 3, 9, 13))
    loss, l1, s, grad = S.hybrid_loss_and_grad(p, t, 0.7)
    assert l1 == pytest.approx(np.abs(p - t).mean(), rel=1e-14)
    assert s == pytest.approx(np.mean([S.ssim_map(p[b], t[b]).mean() for b in range(3)]), rel=1e-14)
    assert loss == pytest.approx(0.7 * l1 + 0.3 * (1 - s), rel=1e-14)
    # central differences of the whole loss (no pixel sits on a sign change of p - t)
    eps = 1e-6
    for ij in [(0, 4, 6), (1, 0, 0), (2, 8, 12), (1, 3, 7)]:
        pp, pm = p.copy(), p.copy()
        pp[ij] += eps
        pm[ij] -= eps
        fd = (S.hybrid_loss_and_grad(pp, t)[0] - S.hybrid_loss_and_grad(pm, t)[0]) / (2 * eps)
        assert grad[ij] == pytest.approx(fd, rel=1e-6, abs=1e-11), ij
    # lambda1 = 1 is the plain l1 loss
    l, _, _, g1 = S.hybrid_loss_and_grad(p, t, 1.0)
    assert l == pytest.approx(l1, rel=1e-15)
    np.testing.assert_allclose(g1, np.sign(p - t) / p.size, rtol=0, atol=0)
