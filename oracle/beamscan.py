"""FP64 reference of the beam-scan spatial spectrum (paper Sec. 3.1).

TEST INFRASTRUCTURE ONLY (see model.py for the import rule).

A sqrt(K) x sqrt(K) planar array with element spacing D; element (m, n),
m, n = 1..sqrt(K), sits at radius r = D sqrt((m-1)^2 + (n-1)^2) and angle
beta = atan2(m - 1, n - 1) (Sec. 3.1, element-position equation). For paths
l = 1..Lp with power coefficient rho_l, azimuth theta_l and elevation phi_l:

  path-length difference   dd_mn(theta, phi) = -r cos(theta - beta) cos(phi)
  phase difference         da_mn(theta, phi) = 2 pi dd_mn(theta, phi) / lambda
                           (eq. for the phase shift; the "mod 2 pi" does not
                           change a complex exponential)
  channel                  h_mn = sum_l rho_l exp(j da_mn(theta_l, phi_l))
                           (eq. for the received signal)
  spectrum                 A(theta, phi) = | (1/K) sum_mn w_mn(theta, phi)
                           exp(j angle(h_mn)) |, w_mn = exp(-j da_mn(theta, phi))
                           (beam-scan equation)

Readings (where the paper is silent): D = lambda / 2 unless given; the grid
samples azimuth theta_x = 2 pi x / W (column x) and elevation phi_y =
(pi / 2) y / H (row y), i.e. 1 degree per pixel at 90 x 360; an element whose
channel is exactly zero (no paths) contributes nothing (its angle is
undefined), so a query without paths renders zero.

Pins: tests/test_oracle_beamscan.py (a single path gives the separable
Dirichlet array factor in closed form, value 1 at its own direction; scaling
all powers leaves A unchanged; one element gives A = 1; no paths give 0).
"""
from __future__ import annotations

import numpy as np


def element_positions(side: int, spacing_over_lambda: float = 0.5):
    """(r / lambda, beta) of the side x side elements, m-major (m, n from 1)."""
    m, n = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    r = spacing_over_lambda * np.sqrt(m ** 2 + n ** 2)
    beta = np.arctan2(m, n)
    return r.ravel().astype(np.float64), beta.ravel().astype(np.float64)


def phase_difference(theta, phi, side: int, spacing_over_lambda: float = 0.5):
    """da_mn(theta, phi) for every element: shape (..., K)."""
    r, beta = element_positions(side, spacing_over_lambda)
    theta = np.asarray(theta, np.float64)[..., None]
    phi = np.asarray(phi, np.float64)[..., None]
    dd = -r * np.cos(theta - beta) * np.cos(phi)  # in wavelengths
    return 2.0 * np.pi * dd


def channel(paths: np.ndarray, count: int, side: int, spacing_over_lambda: float = 0.5) -> np.ndarray:
    """h_mn of one query from its paths (rows of (rho, azimuth, elevation))."""
    p = np.asarray(paths, np.float64)[:count]
    if count == 0:
        return np.zeros(side * side, np.complex128)
    da = phase_difference(p[:, 1], p[:, 2], side, spacing_over_lambda)  # (L, K)
    return (p[:, 0:1] * np.exp(1j * da)).sum(axis=0)


def spectrum(paths: np.ndarray, count: int, H: int, W: int, side: int = 4, spacing_over_lambda: float = 0.5,
             pix=None) -> np.ndarray:
    """A over the H x W grid (row = elevation, column = azimuth) of one query,
    or at the listed pixels pix = (x, y)."""
    K = side * side
    h = channel(paths, count, side, spacing_over_lambda)
    mag = np.abs(h)
    c = np.where(mag > 0, np.exp(1j * np.angle(h)), 0.0)
    if pix is None:
        ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        xs, ys = xs.ravel(), ys.ravel()
    else:
        xs, ys = np.asarray(pix[0]), np.asarray(pix[1])
    theta = 2.0 * np.pi * xs / W
    phi = 0.5 * np.pi * ys / H
    da = phase_difference(theta, phi, side, spacing_over_lambda)  # (P, K)
    A = np.abs((np.exp(-1j * da) * c[None, :]).sum(axis=1)) / K
    return A if pix is not None else A.reshape(H, W)
