"""Pins of the training-step oracles (paper Sec. 4.4: Adam at the hyperparameter
table's learning rates, anneal smoothing) by closed forms."""
import numpy as np
import pytest

from oracle import train as T


def test_adam_first_step_moves_by_lr_sign():
    rng = np.random.default_rng(0)
    g = rng.normal(0, 1, 50)
    p0 = rng.normal(0, 1, 50)
    p1, m, v = T.adam_step(p0, g, np.zeros(50), np.zeros(50), 1e-2, 1)
    # m_hat = g and v_hat = g^2 after one step from zero moments
    np.testing.assert_allclose(p0 - p1, 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-12)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)  # 1 - 0.999 rounds in FP64


def test_adam_constant_gradient_keeps_the_step():
    g = np.array([0.5, -2.0, 3e-3])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 8):
        q, m, v = T.adam_step(p, g, m, v, 8e-3, t)
        # with a constant gradient both bias-corrected moments equal g and g^2 at every step
        np.testing.assert_allclose(p - q, 8e-3 * g / (np.abs(g) + 1e-8), rtol=1e-10)
        p = q


def test_anneal_scale_and_decay():
    tx = np.array([[1.0, 2.0, 0.5], [5.0, 5.5, 2.9]])
    n = np.array([[1.0, -1.0, 0.5], [0.0, 2.0, -3.0]])
    # i = 0, N_s = 8: factor gamma * 2 / 2 = 1 in the unit cube, i.e. the room extent (6, 6, 3) per axis
    np.testing.assert_allclose(T.anneal_tx(tx, n, 0, n_positions=8), tx + n * np.array([6.0, 6.0, 3.0]), rtol=1e-15)
    # half way: half the noise; from tau on: none (the linear factor is clamped at zero)
    np.testing.assert_allclose(T.anneal_tx(tx, n, 5000, n_positions=8), tx + 0.5 * n * np.array([6, 6, 3.0]))
    np.testing.assert_array_equal(T.anneal_tx(tx, n, 10_000, n_positions=8), tx)
    np.testing.assert_array_equal(T.anneal_tx(tx, n, 25_000, n_positions=8), tx)
    # N_s = 1000 positions: sampling interval 2 / 10
    np.testing.assert_allclose(T.anneal_tx(tx, n, 0, n_positions=1000) - tx, 0.2 * n * np.array([6, 6, 3.0]),
                               rtol=1e-12)
