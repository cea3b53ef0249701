"""Pins of the paper-model oracle (Sec. 4.1 GMM spectrum over Cholesky
Gaussians with tanh centres and complex responses; Sec. 4.2 / 6.1 deformation
MLP with skips) by closed forms and structural properties."""
import numpy as np
import pytest

from oracle import model as M
from oracle import paper as P

KEYS = ("center_x", "center_y", "chol_l1", "chol_l2", "chol_l3", "atten_logit", "psi_re", "psi_im")


def _g(rows):
    a = np.asarray(rows, np.float64)
    return {k: np.ascontiguousarray(a[:, j], np.float32) for j, k in enumerate(KEYS)}


def test_centre_map():
    x, y = P.centers([0.0, 40.0, -40.0], [0.0, -40.0, 40.0], 90, 360)
    np.testing.assert_allclose(x, [180.0, 360.0, 0.0], atol=1e-12)
    np.testing.assert_allclose(y, [45.0, 0.0, 90.0], atol=1e-12)


def test_single_gaussian_closed_form():
    H, W = 40, 80
    c = [0.3, -0.2, 2.5, -1.25, 1.75, 0.4, 0.6, -0.8]
    g = _g([c])
    A, re, im, _ = P.render(P.deformed(g, H, W), H, W)
    f = np.float32(c).astype(np.float64)
    mx, my = W / 2 * (np.tanh(f[0]) + 1), H / 2 * (np.tanh(f[1]) + 1)
    l1, l2, l3 = f[2], f[3], f[4]
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    dx, dy = xs.ravel() - mx, ys.ravel() - my
    # Sigma = L L^T = [[l1^2, l1 l2], [l1 l2, l2^2 + l3^2]], det = (l1 l3)^2
    q = ((l2 * l2 + l3 * l3) * dx * dx - 2 * l1 * l2 * dx * dy + l1 * l1 * dy * dy) / (l1 * l3) ** 2
    delta = 1 / (1 + np.exp(-f[5]))
    want = np.where(q <= 9, delta * np.hypot(f[6], f[7]) * np.exp(-q / 2), 0.0)
    np.testing.assert_allclose(A, want, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(re, np.where(q <= 9, f[6] * delta * np.exp(-q / 2), 0.0), rtol=1e-12, atol=1e-15)
    assert A.max() > 0.3


def test_opposite_responses_cancel_and_order_does_not_matter():
    H, W = 32, 64
    a = [0.1, 0.2, 3.0, 1.0, 2.0, 0.5, 0.7, 0.3]
    b = a[:6] + [-0.7, -0.3]
    A, _, _, _ = P.render(P.deformed(_g([a, b]), H, W), H, W)
    np.testing.assert_allclose(A, 0.0, atol=1e-15)
    rng = np.random.default_rng(0)
    rows = np.stack([rng.normal(0, 0.8, 40), rng.normal(0, 0.8, 40), rng.uniform(1, 5, 40), rng.normal(0, 1, 40),
                     rng.uniform(1, 5, 40), rng.normal(0, 1, 40), rng.normal(0, 1, 40), rng.normal(0, 1, 40)], 1)
    A1, _, _, _ = P.render(P.deformed(_g(rows), H, W), H, W)
    A2, _, _, _ = P.render(P.deformed(_g(rows[rng.permutation(40)]), H, W), H, W)
    np.testing.assert_allclose(A1, A2, rtol=1e-12, atol=1e-14)
    # a common phase on every response leaves the magnitude unchanged
    ph = 0.77
    rot = rows.copy()
    rot[:, 6] = np.float32(np.cos(ph) * rows[:, 6] - np.sin(ph) * rows[:, 7])
    rot[:, 7] = np.float32(np.sin(ph) * rows[:, 6] + np.cos(ph) * rows[:, 7])
    A3, _, _, _ = P.render(P.deformed(_g(rot), H, W), H, W)
    np.testing.assert_allclose(A3, A1, rtol=1e-6, atol=1e-7)  # the rotated responses are rounded to FP32


def test_degenerate_and_deformation():
    H, W = 16, 32
    g = _g([[0.0, 0.0, 0.0, 1.0, 2.0, 1.0, 1.0, 0.0], [0.0, 0.0, 2.0, 1.0, 0.0, 1.0, 1.0, 0.0]])
    A, _, _, _ = P.render(P.deformed(g, H, W), H, W)
    np.testing.assert_array_equal(A, 0.0)
    # residuals: the centre moves by d_mu pixels, psi by d_psi, delta by d_delta after the gate
    g = _g([[0.0, 0.0, 2.0, 0.0, 2.0, 0.0, 1.0, 0.0]])
    d = np.array([[3.0, -2.0, 0.5, 0.25, 0.1]])
    dg = P.deformed(g, H, W, d)
    assert dg["x"][0] == pytest.approx(19.0) and dg["y"][0] == pytest.approx(6.0)
    assert dg["wr"][0] == pytest.approx(1.5 * 0.6) and dg["wi"][0] == pytest.approx(0.25 * 0.6)


def test_mlp_shapes_and_parameter_count():
    shapes = P.layer_shapes()
    assert shapes[0] == (156, 81) and shapes[2] == (156, 237) and shapes[1] == (156, 156)
    assert [s[1] for s in shapes] == [81, 156, 237, 156, 237, 156, 237, 156, 156] and shapes[-1] == (5, 156)
    assert sum(o * i + o for o, i in shapes) == 222_929


@pytest.mark.parametrize("skip", [3, 5, 7])
def test_mlp_skip_carries_the_input_after_the_hidden_state(skip):
    # every layer before `skip` is zero, so the hidden state entering it is 0 and only the concatenated input
    # [h, x] can reach the output: layer `skip` copies x[j] (columns 156 + j) to unit j, later layers pass units
    # through, and the output reads units 0 and 3: ReLU(mu_hat_x) and ReLU(sin(pi mu_hat_y))
    shapes = P.layer_shapes()
    Ws = [np.zeros(s) for s in shapes]
    bs = [np.zeros(s[0]) for s in shapes]
    for j in range(81):
        Ws[skip - 1][j, 156 + j] = 1.0
    for l in range(skip, 8):
        Ws[l][:, :156] = np.eye(156)
    Ws[8][0, 0] = 1.0
    Ws[8][1, 3] = 1.0
    bs[8][4] = 0.25
    rng = np.random.default_rng(skip)
    g = _g(np.stack([rng.normal(0, 1, 30), rng.normal(0, 1, 30)] + [np.ones(30)] * 6, 1))
    out = P.mlp_forward(P.features(g, [1.0, 2.0, 0.5], 90, 360), Ws, bs)
    x, y = P.centers(np.float32(g["center_x"]).astype(np.float64), np.float32(g["center_y"]).astype(np.float64),
                     90, 360)
    np.testing.assert_allclose(out[:, 0], x / 360, rtol=1e-14)
    np.testing.assert_allclose(out[:, 1], np.maximum(np.sin(np.pi * y / 90), 0.0), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(out[:, 4], 0.25)
    # the same weights with the input entering at any other layer would give zeros: check one
    if skip != 3:
        Ws2 = [w.copy() for w in Ws]
        Ws2[skip - 1][:, 156:] = 0.0
        assert np.abs(P.mlp_forward(P.features(g, [1.0, 2.0, 0.5], 90, 360), Ws2, bs)[:, :2]).max() == 0.0


def test_feature_layout():
    g = _g([[0.0, 0.0, 1, 0, 1, 0, 1, 0]])
    f = P.features(g, [3.0, 3.0, 1.5], 90, 360)
    assert f.shape == (1, 81)
    # the centre maps to (180, 45): mu_hat = (0.5, 0.5); the position to the room's centre: s_hat = (0.5, 0.5, 0.5)
    np.testing.assert_allclose(f[0, :2], [0.5, 0.5])
    np.testing.assert_allclose(f[0, 2:4], np.sin(np.pi * 0.5))  # band 0 sines
    np.testing.assert_allclose(f[0, 42:45], [0.5, 0.5, 0.5])
    assert M.posenc(np.zeros((1, 2)), 10).shape == (1, 42)
