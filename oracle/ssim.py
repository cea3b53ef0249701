"""FP64 reference of the training objective's SSIM term and of the hybrid loss
(paper Sec. 4.4, the hybrid-loss equation: L = l1 * |A_hat - A|_1 +
(1 - l1) * (1 - SSIM(A_hat, A)), l1 = 0.7 in the hyperparameter table).

TEST INFRASTRUCTURE ONLY (see model.py for the import rule).

The paper names SSIM without its parameters. Reading used (the structural
similarity index of Wang et al. as 3DGS-style trainers compute it): an 11 x 11
Gaussian window of standard deviation 1.5 normalised to sum 1, local
statistics by weighted window sums with zero padding so the map has the image's
size, C1 = 0.01^2 and C2 = 0.03^2 (data range 1), and the loss's SSIM is the
mean of the map over every pixel of every spectrum of the batch:

  mu_x = w * x,  sigma_x^2 = w * x^2 - mu_x^2,  sigma_xy = w * (x y) - mu_x mu_y
  S = (2 mu_x mu_y + C1)(2 sigma_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2))

The l1 term is the mean absolute difference over the batch (sign(0) = 0 in its
gradient). The gradient with respect to the prediction is the chain rule of
these formulas written out (the window sums are linear, so each local statistic
sends its derivative back through the same window).

Pins: tests/test_oracle_ssim.py (identical images give 1; symmetry; constant
images in the interior give the closed form; a one-pixel image gives the
closed form with the window's centre weight; central differences of the
gradient).
"""
from __future__ import annotations

import numpy as np

WIN = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2
LAMBDA1 = 0.7


def window() -> np.ndarray:
    """The 11 x 11 Gaussian window (outer product of the normalised 1D Gaussian)."""
    r = np.arange(WIN) - WIN // 2
    g = np.exp(-(r.astype(np.float64) ** 2) / (2.0 * SIGMA ** 2))
    g /= g.sum()
    return np.outer(g, g)


def _wsum(img: np.ndarray) -> np.ndarray:
    """Window sum at every pixel with zero padding: out[i, j] = sum_ab w[a, b] img[i + a - 5, j + b - 5]."""
    H, W = img.shape
    h = WIN // 2
    pad = np.zeros((H + 2 * h, W + 2 * h))
    pad[h:h + H, h:h + W] = img
    w = window()
    out = np.zeros((H, W))
    for a in range(WIN):
        for b in range(WIN):
            out += w[a, b] * pad[a:a + H, b:b + W]
    return out


def ssim_map(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = _wsum(x), _wsum(y)
    sxx = _wsum(x * x) - mx * mx
    syy = _wsum(y * y) - my * my
    sxy = _wsum(x * y) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def ssim_and_grad(x: np.ndarray, y: np.ndarray) -> tuple:
    """(mean SSIM over the image, d mean / d x) for one H x W image pair."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    n = x.size
    mx, my = _wsum(x), _wsum(y)
    exx, eyy, exy = _wsum(x * x), _wsum(y * y), _wsum(x * y)
    vx, vy, cxy = exx - mx * mx, eyy - my * my, exy - mx * my
    N1, N2 = 2 * mx * my + C1, 2 * cxy + C2
    D1, D2 = mx * mx + my * my + C1, vx + vy + C2
    S = N1 * N2 / (D1 * D2)
    # derivatives of S with respect to the window sums mu_x, E[x^2], E[x y] (mu_y, E[y^2] belong to the target)
    # through N1 (d/dmu_x = 2 mu_y), N2 (d/dmu_x = -2 mu_y, d/dE[xy] = 2), D1 (d/dmu_x = 2 mu_x),
    # D2 (d/dmu_x = -2 mu_x, d/dE[x^2] = 1)
    dS_dm = (2 * my * N2 - 2 * my * N1) / (D1 * D2) - 2 * mx * S / D1 + 2 * mx * S / D2
    dS_dexx = -S / D2
    dS_dexy = 2 * N1 / (D1 * D2)
    # each window sum at p depends on x(q) with weight w(p - q): send back through the same (symmetric) window
    g = (_wsum(dS_dm) + 2.0 * x * _wsum(dS_dexx) + y * _wsum(dS_dexy)) / n
    return float(S.mean()), g


def hybrid_loss_and_grad(pred: np.ndarray, target: np.ndarray, lambda1: float = LAMBDA1) -> tuple:
    """Hybrid loss over a batch (B x H x W): lambda1 * mean |pred - target| + (1 - lambda1) * (1 - mean SSIM),
    the SSIM averaged over every pixel of every spectrum. Returns (loss, l1, ssim, d loss / d pred)."""
    pred = np.asarray(pred, np.float64)
    target = np.asarray(target, np.float64)
    B = pred.shape[0]
    count = pred.size
    l1 = float(np.abs(pred - target).sum() / count)
    s_tot = 0.0
    grad = np.zeros_like(pred)
    for b in range(B):
        s, g = ssim_and_grad(pred[b], target[b])
        s_tot += s / B
        grad[b] = -(1.0 - lambda1) * g / B
    grad += lambda1 * np.sign(pred - target) / count
    loss = lambda1 * l1 + (1.0 - lambda1) * (1.0 - s_tot)
    return loss, l1, s_tot, grad
