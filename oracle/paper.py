"""FP64 reference of the paper's own spectrum model (Sec. 4.1 and 4.2): the
order-free GMM sum of complex responses over Cholesky-parameterised 2D
Gaussians with tanh-normalised centres, deformed by the paper's MLP.

TEST INFRASTRUCTURE ONLY (see model.py for the import rule).

Per Gaussian n (raw parameters, pixel units where they are lengths):
  centre   x = (W / 2)(tanh(c_x) + 1), y = (H / 2)(tanh(c_y) + 1): the
           hyperbolic normalisation of Sec. 4.1 maps the azimuth into
           [0, 2 pi] and the elevation into [0, pi / 2]; each range is the
           grid's extent along that axis (the paper's symbols for the two
           angles are swapped between Sec. 3 and Sec. 4; each axis is mapped
           onto its own grid here)
  Sigma    = L L^T with L = [[l1, 0], [l2, l3]] (Cholesky factor, Sec. 3.2)
  delta    = sigmoid(a), the attenuation gate (Sec. 4.1)
  psi      = (psi_re, psi_im), the complex signal response (Sec. 4.1)
Kernel weight K_n(p) = delta_n exp(-q/2), q = d^T Sigma^-1 d, d = p - centre
(Sec. 4.1 kernel-weight equation), and the spectrum (Sec. 4.1 rasterization
equation; Sec. 6.1: real and imaginary parts as two channels, then the
magnitude) A(p) = | sum_n psi_n K_n(p) |. Reading: the sum runs over the
Gaussians whose q <= 9 at p (the 3-sigma support the tile binning uses); there
is no ordering, no opacity clamp, no skip and no termination. Degenerate
(l1 l3 = 0) or non-finite Gaussians take no part.

Deformation (Sec. 4.2): residuals (d_mu_x, d_mu_y, d_psi_re, d_psi_im,
d_delta) = F_theta(gamma(mu_hat), gamma(s_hat)) with 10 frequency bands for the
centre and 6 for the position (Sec. 6.1; gamma as in model.posenc, identity
term included: 2 * 21 + 3 * 13 = 81 inputs, mu_hat = (x / W, y / H) of the
canonical centre, s_hat the position in the room's unit cube). Deformed:
centre + d_mu (pixels), psi + d_psi, delta = sigmoid(a) + d_delta (added after
the gate, as the residual equations write it); the covariance is not deformed.
MLP (Sec. 6.1): eight layers of width 156 with ReLU and skip connections every
two layers -- read as the input features concatenated after the hidden state
entering layers 3, 5 and 7 ([h, x]) -- and a linear output layer of 5.

Pins: tests/test_oracle_paper.py.
"""
from __future__ import annotations

import numpy as np

from . import model as M

CENTER_BANDS = 10
TX_BANDS = 6
WIDTH = 156
N_LAYERS = 8
SKIP_LAYERS = (3, 5, 7)  # 1-based layers whose input is [h, x]
N_IN = 2 * (2 * CENTER_BANDS + 1) + 3 * (2 * TX_BANDS + 1)  # 81
N_OUT = 5
Q_MAX = 9.0


def layer_shapes():
    """(out, in) of the 8 hidden layers and the output layer."""
    shapes = []
    for l in range(1, N_LAYERS + 1):
        if l == 1:
            k = N_IN
        elif l in SKIP_LAYERS:
            k = WIDTH + N_IN
        else:
            k = WIDTH
        shapes.append((WIDTH, k))
    shapes.append((N_OUT, WIDTH))
    return shapes


def centers(cx, cy, H, W):
    return 0.5 * W * (np.tanh(np.asarray(cx, np.float64)) + 1.0), 0.5 * H * (np.tanh(np.asarray(cy, np.float64)) + 1.0)


def mlp_forward(x, Ws, bs):
    """FP64 forward of the paper MLP; x (P, 81) -> (P, 5)."""
    x = np.asarray(x, np.float64)
    h = x
    for l in range(1, N_LAYERS + 1):
        inp = np.concatenate([h, x], axis=1) if l in SKIP_LAYERS else h
        h = np.maximum(inp @ np.asarray(Ws[l - 1], np.float64).T + np.asarray(bs[l - 1], np.float64), 0.0)
    return h @ np.asarray(Ws[N_LAYERS], np.float64).T + np.asarray(bs[N_LAYERS], np.float64)


def features(g: dict, tx, H, W, room=M.DEFAULT_ROOM):
    """(P, 81) MLP inputs of every Gaussian for one position."""
    x, y = centers(g["center_x"], g["center_y"], H, W)
    mu_hat = np.stack([x / W, y / H], axis=1)
    fm = M.posenc(mu_hat, CENTER_BANDS)
    fs = M.posenc(M.normalize_tx(np.asarray(tx, np.float64), room)[None, :], TX_BANDS)
    return np.concatenate([fm, np.repeat(fs, len(x), axis=0)], axis=1)


def deformed(g: dict, H, W, delta=None):
    """Deformed per-Gaussian quantities: centre (x, y), Sigma^-1 entries, complex weight psi * delta, live mask."""
    f64 = lambda k: np.asarray(g[k], np.float32).astype(np.float64)
    x, y = centers(f64("center_x"), f64("center_y"), H, W)
    l1, l2, l3 = f64("chol_l1"), f64("chol_l2"), f64("chol_l3")
    dl = 1.0 / (1.0 + np.exp(-f64("atten_logit")))
    pr, pi = f64("psi_re"), f64("psi_im")
    if delta is not None:
        d = np.asarray(delta, np.float64)
        x, y = x + d[:, 0], y + d[:, 1]
        pr, pi = pr + d[:, 2], pi + d[:, 3]
        dl = dl + d[:, 4]
    sxx, sxy, syy = l1 * l1, l1 * l2, l2 * l2 + l3 * l3
    det = sxx * syy - sxy * sxy
    with np.errstate(divide="ignore", invalid="ignore"):
        ixx, ixy, iyy = syy / det, -sxy / det, sxx / det
    live = (l1 * l3 != 0) & np.isfinite(x) & np.isfinite(y) & np.isfinite(ixx) & np.isfinite(ixy) & \
        np.isfinite(iyy) & np.isfinite(pr) & np.isfinite(pi) & np.isfinite(dl)
    return dict(x=x, y=y, ixx=ixx, ixy=ixy, iyy=iyy, wr=pr * dl, wi=pi * dl, live=live, sxx=sxx, syy=syy)


def render(dg: dict, H, W, pix=None, margin=1e-4, chunk=4096):
    """GMM sum at the listed pixels (default the full grid): (A, re, im, bound) with bound the sum of |weight|
    e^{-q/2} over Gaussians whose q lies within `margin` (relative) of the cutoff -- the most a decision taken the
    other way in FP32 can move A."""
    if pix is None:
        pix = M.full_grid(H, W)
    px, py = np.asarray(pix[0], np.float64), np.asarray(pix[1], np.float64)
    L = dg["live"]
    x, y, ixx, ixy, iyy, wr, wi = (dg[k][L] for k in ("x", "y", "ixx", "ixy", "iyy", "wr", "wi"))
    re = np.zeros(len(px))
    im = np.zeros(len(px))
    bound = np.zeros(len(px))
    for s in range(0, len(px), chunk):
        dx = px[s:s + chunk, None] - x[None, :]
        dy = py[s:s + chunk, None] - y[None, :]
        q = ixx * dx * dx + 2.0 * ixy * dx * dy + iyy * dy * dy
        e = np.exp(-0.5 * q)
        inside = q <= Q_MAX
        re[s:s + chunk] = np.where(inside, wr * e, 0.0).sum(axis=1)
        im[s:s + chunk] = np.where(inside, wi * e, 0.0).sum(axis=1)
        near = np.abs(q - Q_MAX) <= margin * Q_MAX
        bound[s:s + chunk] = np.where(near, np.hypot(wr, wi) * e, 0.0).sum(axis=1)
    return np.hypot(re, im), re, im, bound


def at_grid(dg: dict, sx: float, sy: float) -> dict:
    """Deformed Gaussians on another resolution of the same field of view: coordinates scale by (sx, sy), so the
    centres do and Sigma' = S Sigma S."""
    d2 = dict(dg)
    d2["x"], d2["y"] = dg["x"] * sx, dg["y"] * sy
    d2["ixx"], d2["ixy"], d2["iyy"] = dg["ixx"] / (sx * sx), dg["ixy"] / (sx * sy), dg["iyy"] / (sy * sy)
    d2["sxx"], d2["syy"] = dg["sxx"] * sx * sx, dg["syy"] * sy * sy
    return d2


def render_query(g: dict, H, W, mlp=None, tx=None, room=M.DEFAULT_ROOM, pix=None, grid=None):
    """(A, re, im, bound, delta) of one query: deformed by the MLP ((Ws, bs) lists) when given; grid = (H', W')
    renders another resolution of the same field of view."""
    delta = None
    if mlp is not None:
        delta = mlp_forward(features(g, tx, H, W, room), mlp[0], mlp[1])
    dg = deformed(g, H, W, delta)
    if grid is not None and tuple(grid) != (H, W):
        dg = at_grid(dg, grid[1] / W, grid[0] / H)
        H, W = grid
    A, re, im, bound = render(dg, H, W, pix)
    return A, re, im, bound, delta
