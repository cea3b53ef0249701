"""FP64 reference of the RSSI head (paper Sec. 7.2, RSSI case study).

TEST INFRASTRUCTURE ONLY (see model.py for the import rule).

The head pools the rendered spectrum map by a global average over elevation
and azimuth into one value per query: rssi = (1 / (H W)) sum_{y, x} A(y, x).
The spectrum is the oracle's brute-force render (model.render_query); its
gradient with respect to any parameter is that of sum_p w_p A_p with every
pixel weight w_p = dL/drssi / (H W), which grad.loss_and_grad takes as pixel
weights.

Pins: tests/test_oracle_rssi.py (a 1 x 1 grid gives the pixel itself;
Gaussians whose 3-sigma boxes share no pixel add; moving a Gaussian that lies
wholly inside the grid by whole pixels leaves the value unchanged; an empty
scene gives 0).
"""
from __future__ import annotations

import numpy as np

from . import model as M


def pool(spectrum: np.ndarray) -> float:
    """Global average of one H x W spectrum (FP64)."""
    a = np.asarray(spectrum, np.float64)
    return float(a.sum() / a.size)


def rssi_query(scene: M.Scene, mlp, tx, bf16: bool = False, delta=None) -> tuple:
    """(rssi, RenderResult) of one query: the oracle's spectrum over the full grid, pooled."""
    res, _, _, _ = M.render_query(scene, mlp, tx, bf16=bf16, delta=delta)
    return pool(res.C), res


def pixel_weights(grad_rssi: float, H: int, W: int) -> np.ndarray:
    """Pixel weights whose weighted spectrum sum has the gradient of grad_rssi * rssi."""
    return np.full(H * W, grad_rssi / (H * W), np.float64)
