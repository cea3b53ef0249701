"""Pins of the oracle's positional encoding (Sec. 4.2, eq. posenc), its
deformation MLP (Sec. 4.2) and its bfloat16 rounding."""
import math

import numpy as np
import pytest
import torch

from oracle import model as M
from paper_2506_12787_amd import synth


def test_posenc_width_matches_d_2L_plus_1():
    assert M.posenc(np.zeros(2), 6).shape == (26,)
    assert M.posenc(np.zeros(3), 10).shape == (63,)


def test_posenc_special_values():
    r2 = math.sqrt(0.5)
    g = M.posenc(np.array([0.5, 0.25]), 2)
    # [v | sin(pi v) | sin(2 pi v) | cos(pi v) | cos(2 pi v)], components in order
    expect = [0.5, 0.25, 1.0, r2, 0.0, 1.0, 0.0, r2, -1.0, 0.0]
    np.testing.assert_allclose(g, expect, atol=1e-15)
    g0 = M.posenc(np.zeros(3), 10)
    np.testing.assert_array_equal(g0, np.r_[np.zeros(3 + 30), np.ones(30)])


def _onehot_mlp(j, d_in=89, hidden=8, n_hidden=4):
    W = [np.zeros((hidden, d_in))] + [np.eye(hidden) for _ in range(n_hidden - 1)] + [np.zeros((7, hidden))]
    W[0][0, j] = 1.0
    W[-1][3, 0] = 2.0
    b = [np.zeros(hidden) for _ in range(n_hidden)] + [np.zeros(7)]
    b[-1][6] = 0.25
    return M.MLP(W, b)


def test_mlp_onehot_routes_one_feature():
    # unit 0 copies input feature j through the ReLU chain; output 3 = 2 relu(x_j)
    xm = M.posenc(np.array([[0.5, 0.25]]), 6)
    xs = M.posenc(np.array([0.5, 0.0, 1.0]), 10)
    # feature 26 + 3 = sin(pi * 0.5) = 1 ; feature 26 + 3 + 3*1 + 2 = sin(2 pi * 1.0) ~ 0
    out, _, _ = M.mlp_forward(xm, xs, _onehot_mlp(26 + 3))
    np.testing.assert_allclose(out[0], [0, 0, 0, 2.0, 0, 0, 0.25], atol=1e-15)
    # feature 26 + 33 = cos(pi * 0.5) ~ 0 ; 26 + 34 = cos(pi * 0) = 1; 26+35 = cos(pi)= -1 -> relu 0
    out, _, _ = M.mlp_forward(xm, xs, _onehot_mlp(26 + 34))
    assert out[0, 3] == pytest.approx(2.0, abs=1e-15)
    out, _, _ = M.mlp_forward(xm, xs, _onehot_mlp(26 + 35))
    assert out[0, 3] == 0.0
    # a mean feature: index 2 = sin(pi * mu_hat_x) = 1 at mu_hat_x = 0.5
    out, _, _ = M.mlp_forward(xm, xs, _onehot_mlp(2))
    assert out[0, 3] == pytest.approx(2.0, abs=1e-15)


def test_mlp_is_affine_without_relu_activity():
    # all-positive weights and inputs keep every ReLU open: then F is affine
    rng = np.random.default_rng(0)
    W = [rng.uniform(0, 1, (16, 89))] + [rng.uniform(0, 1, (16, 16)) for _ in range(3)] + [rng.uniform(0, 1, (7, 16))]
    b = [rng.uniform(0, 1, 16) for _ in range(4)] + [rng.uniform(-1, 1, 7)]
    mlp = M.MLP(W, b)
    xa, xb = rng.uniform(0, 1, (1, 26)), rng.uniform(0, 1, (1, 26))
    s = rng.uniform(0, 1, 63)
    f = lambda x: M.mlp_forward(x, s, mlp)[0]
    z = np.zeros((1, 26))
    np.testing.assert_allclose(f(xa + xb) - f(xa) - f(xb) + f(z), 0, atol=1e-8 * np.abs(f(xa)).max())


def test_zero_weights_give_zero_residuals_and_static_render():
    H, W = 24, 40
    g = synth.gaussians(80, H, W, seed=3)
    s = M.Scene.from_arrays(g, H, W)
    Ws, bs = synth.mlp_weights(seed=4, hidden=32)
    mlp = M.MLP([np.zeros_like(w, dtype=np.float64) for w in Ws], [np.zeros_like(b, dtype=np.float64) for b in bs])
    tx = synth.tx_positions(1, seed=5)[0]
    r_def, _, _, d = M.render_query(s, mlp, tx)
    r_sta, _, _, _ = M.render_query(s, None, None)
    assert np.all(d == 0)
    np.testing.assert_array_equal(r_def.C, r_sta.C)


def test_bf16_round_matches_torch_conversion():
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e-3, 2000), rng.uniform(-300, 300, 2000)])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16_round(x32.astype(np.float64)), ref)
    # exact ties round to even
    assert M.bf16_round(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert M.bf16_round(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6


def test_bf16_mlp_equals_fp64_mlp_on_bf16_exact_operands():
    # signed-permutation hidden layers and +-1/2 one-feature first-layer rows keep
    # every operand and activation exactly representable in bfloat16
    rng = np.random.default_rng(8)
    hdim = 16
    W1 = np.zeros((hdim, 89))
    for u in range(hdim):
        W1[u, rng.integers(0, 26)] = rng.choice([0.5, 1.0])
    W = [W1]
    for _ in range(3):
        P = np.eye(hdim)[rng.permutation(hdim)]
        W.append(P)
    W.append(rng.integers(-1, 2, (7, hdim)).astype(float))
    b = [np.zeros(hdim) for _ in range(4)] + [np.zeros(7)]
    mlp = M.MLP(W, b)
    xm = np.round(M.posenc(np.array([[0.5, 0.0], [0.0, 0.5], [0.25, 0.75]]), 6) * 4) / 4
    xs = M.posenc(np.array([0.3, 0.5, 0.1]), 10)  # TX part has zero weights here
    a = M.mlp_forward(xm, xs, mlp, bf16=True)[0]
    e = M.mlp_forward(xm, xs, mlp)[0]
    np.testing.assert_array_equal(a, e)
    assert np.abs(e).max() > 0
