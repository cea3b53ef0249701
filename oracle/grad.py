"""FP64 analytic gradient of the L1 training loss through compositing, the
covariance, the deformation and the deformation MLP; plus the finite-difference
harness that pins it.

TEST INFRASTRUCTURE ONLY (see oracle/model.py for the import rule).

Loss (Sec. 4.4, the L1 term of the hybrid loss): mean over B*H*W pixels of
|A_hat - A|, with sign(0) = 0. Every discrete decision (3-sigma cutoff, alpha
skip, transmittance floor, alpha clamp) is held at its FP64 outcome; where the
0.99 clamp is active the derivative through opacity and q is zero.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import model as M


def _pixel_weights(C, target, count):
    return np.sign(C - target) / float(count)


def raster_grad(rg: dict, order, pix, w, flags_out=None):
    """d(sum_p w_p C_p) / d(mx, my, ixx, ixy, iyy, opacity, amp) per Gaussian.
    flags_out (int8 array of n), if given, receives the near-threshold marks."""
    lib = M._raster()
    n = len(rg["mx"])
    grad = np.zeros((n, 7))
    order = np.ascontiguousarray(order, np.int64)
    px = np.ascontiguousarray(pix[0], np.int32)
    py = np.ascontiguousarray(pix[1], np.int32)
    w = np.ascontiguousarray(w, np.float64)
    consts = np.array([M.ALPHA_MAX, M.ALPHA_MIN, M.T_MIN, M.Q_MAX], np.float64)
    P = M._ptr
    marg = np.array(M.DEFAULT_MARGINS, np.float64)
    lib.oracle_grad(n, P(rg["mx"]), P(rg["my"]), P(rg["ixx"]), P(rg["ixy"]), P(rg["iyy"]), P(rg["op"]),
                    P(rg["amp"]), P(rg["live"]), P(order), P(consts), P(marg), len(px), P(px), P(py), P(w), P(grad),
                    None if flags_out is None else P(flags_out))
    return grad


def chain_to_params(g: dict, rg: dict, graster: np.ndarray) -> np.ndarray:
    """Map per-Gaussian raster gradients to the 7 deformed parameters
    (mx, my, lsx, lsy, rot, logit, amp)."""
    ixx, ixy, iyy = rg["ixx"], rg["ixy"], rg["iyy"]
    gixx, gixy, giyy = graster[:, 2], graster[:, 3], graster[:, 4]
    # matrix gradient of the inverse (off-diagonal entries each get half)
    Ga = np.stack([np.stack([gixx, 0.5 * gixy], -1), np.stack([0.5 * gixy, giyy], -1)], -2)
    I = np.stack([np.stack([ixx, ixy], -1), np.stack([ixy, iyy], -1)], -2)
    # I = Sigma^-1  =>  dL/dSigma = -I (dL/dI) I
    GS = -np.einsum("nab,nbc,ncd->nad", I, Ga, I)
    c, s = np.cos(g["rot"]), np.sin(g["rot"])
    ex, ey = np.exp(2.0 * g["lsx"]), np.exp(2.0 * g["lsy"])
    dS = {
        "lsx": (2 * c * c * ex, 2 * c * s * ex, 2 * s * s * ex),
        "lsy": (2 * s * s * ey, -2 * c * s * ey, 2 * c * c * ey),
        "rot": (2 * c * s * (ey - ex), (c * c - s * s) * (ex - ey), 2 * c * s * (ex - ey)),
    }
    out = np.zeros((len(c), 7))
    live = rg["live"].astype(bool)
    out[:, 0] = graster[:, 0]
    out[:, 1] = graster[:, 1]
    for j, k in ((2, "lsx"), (3, "lsy"), (4, "rot")):
        dxx, dxy, dyy = dS[k]
        out[:, j] = GS[:, 0, 0] * dxx + 2.0 * GS[:, 0, 1] * dxy + GS[:, 1, 1] * dyy
    op = g["opacity"]
    out[:, 5] = graster[:, 5] * op * (1.0 - op)
    out[:, 6] = graster[:, 6]
    out[~live] = 0.0
    return out


def mlp_backward(x_mean, x_tx, mlp: M.MLP, dout):
    """Backward of F_theta for rows sharing one TX feature vector. Returns
    (dW list, db list, d x_mean)."""
    out, pres, acts = M.mlp_forward(x_mean, x_tx, mlp)
    L = mlp.n_layers
    dW = [None] * L
    db = [None] * L
    d = dout
    for l in range(L - 1, 0, -1):
        h = acts[l - 1]
        dW[l] = d.T @ h
        db[l] = d.sum(0)
        dh = d @ mlp.W[l]
        d = dh * (pres[l - 1] > 0)
    x_full = np.concatenate([x_mean, np.broadcast_to(np.atleast_2d(x_tx), (x_mean.shape[0], x_tx.shape[-1]))], -1)
    dW[0] = d.T @ x_full
    db[0] = d.sum(0)
    dxm = d @ mlp.W[0][:, : x_mean.shape[1]]
    return dW, db, dxm


def posenc_backward(v, L, dgamma):
    """d/dv of sum(dgamma * gamma(v)) for gamma of eq. (posenc)."""
    v = np.asarray(v, np.float64)
    d = v.shape[-1]
    out = dgamma[..., :d].copy()
    for k in range(L):
        f = (2.0 ** k) * np.pi
        out += dgamma[..., d * (1 + k): d * (2 + k)] * f * np.cos(f * v)
        out -= dgamma[..., d * (1 + L + k): d * (2 + L + k)] * f * np.sin(f * v)
    return out


def loss_and_grad(scene: M.Scene, mlp: M.MLP | None, txs, targets, room=M.DEFAULT_ROOM, stop_grad_pos=False,
                  pixel_weights=None):
    """L1 loss over a batch of queries and its FP64 gradient.

    Returns (loss, grads) where grads has 'base' (n, 7) for
    (mx, my, lsx, lsy, rot, logit, amp) and, with an MLP, 'W'/'b' lists.
    With pixel_weights (one array of H*W per query) the objective is instead
    sum_b sum_p w_bp C_bp, and the returned loss is that sum."""
    B = len(txs)
    H, W = scene.H, scene.W
    count = B * H * W
    pix = M.full_grid(H, W)
    order = M.depth_order(scene.depth)
    gbase = np.zeros((scene.n, 7))
    gflag = np.zeros(scene.n, np.int8)
    gW = [np.zeros_like(w) for w in mlp.W] if mlp is not None else None
    gb = [np.zeros_like(b) for b in mlp.b] if mlp is not None else None
    loss = 0.0
    xm = M.posenc(M.normalize_mean(scene.mx, scene.my, H, W), M.MEAN_BANDS) if mlp is not None else None
    for b in range(B):
        delta = M.deltas(scene, mlp, txs[b], room) if mlp is not None else None
        g = M.deform(scene, delta)
        rg = M.gaussians_for_raster(g, scene.depth)
        res = M.composite(rg, order, pix[0], pix[1], margins=None)
        if pixel_weights is not None:
            w = np.asarray(pixel_weights[b], np.float64).ravel()
            loss += float((w * res.C).sum())
        else:
            t = np.asarray(targets[b], np.float64).ravel()
            loss += np.abs(res.C - t).sum() / count
            w = _pixel_weights(res.C, t, count)
        fl = np.zeros(scene.n, np.int8)
        gr = raster_grad(rg, order, pix, w, fl)
        gflag |= fl
        gp = chain_to_params(g, rg, gr)
        gbase += gp
        if mlp is not None:
            xs = M.posenc(M.normalize_tx(txs[b], room), M.TX_BANDS)
            dW, db, dxm = mlp_backward(xm, xs, mlp, gp)
            for l in range(mlp.n_layers):
                gW[l] += dW[l]
                gb[l] += db[l]
            mu_hat = M.normalize_mean(scene.mx, scene.my, H, W)
            dmu_hat = posenc_backward(mu_hat, M.MEAN_BANDS, dxm)
            gbase[:, 0] += dmu_hat[:, 0] / W
            gbase[:, 1] += dmu_hat[:, 1] / H
    if stop_grad_pos:
        gbase[:, 0:2] = 0.0
    return loss, dict(base=gbase, W=gW, b=gb, flagged=gflag.astype(bool))


def loss_only(scene: M.Scene, mlp, txs, targets, room=M.DEFAULT_ROOM):
    """L1 loss plus, per query, the decision signatures, residual signs and MLP
    ReLU patterns used by the finite-difference stability filter."""
    B = len(txs)
    H, W = scene.H, scene.W
    count = B * H * W
    pix = M.full_grid(H, W)
    loss = 0.0
    sigs, signs = [], []
    xm = M.posenc(M.normalize_mean(scene.mx, scene.my, H, W), M.MEAN_BANDS) if mlp is not None else None
    for b in range(B):
        delta = None
        if mlp is not None:
            xs = M.posenc(M.normalize_tx(txs[b], room), M.TX_BANDS)
            delta, pres, _ = M.mlp_forward(xm, xs, mlp)
            signs.append(np.concatenate([(p > 0).ravel() for p in pres]).astype(np.float64))
        res, _, _, _ = M.render_query(scene, mlp, txs[b], room, pix=pix, margins=None, delta=delta)
        t = np.asarray(targets[b], np.float64).ravel()
        loss += np.abs(res.C - t).sum() / count
        sigs.append(res.sig.copy())
        signs.append(np.sign(res.C - t))
    return loss, np.concatenate(sigs), np.concatenate(signs)


def held_state(scene: M.Scene, mlp, txs, targets, room=M.DEFAULT_ROOM):
    """Decisions of the base point, per query: the compositor's inputs (which fix
    every cutoff, skip, clamp and stop decision), the MLP's ReLU patterns and
    the residual signs."""
    H, W = scene.H, scene.W
    pix = M.full_grid(H, W)
    order = M.depth_order(scene.depth)
    xm = M.posenc(M.normalize_mean(scene.mx, scene.my, H, W), M.MEAN_BANDS) if mlp is not None else None
    st = []
    for b in range(len(txs)):
        masks, delta = None, None
        if mlp is not None:
            xs = M.posenc(M.normalize_tx(txs[b], room), M.TX_BANDS)
            delta, pres, _ = M.mlp_forward(xm, xs, mlp)
            masks = [p > 0 for p in pres]
        g = M.deform(scene, delta)
        rg = M.gaussians_for_raster(g, scene.depth)
        res = M.composite(rg, order, pix[0], pix[1], margins=None)
        sign = np.sign(res.C - np.asarray(targets[b], np.float64).ravel())
        st.append(dict(rg=rg, masks=masks, sign=sign))
    return st


def loss_held(scene: M.Scene, mlp, txs, targets, state, room=M.DEFAULT_ROOM):
    """The L1 loss with every discrete decision held at the base point `state`
    (held_state): compositing decisions, ReLU patterns and residual signs, so
    the loss is sum_p sign0_p (C_p - target_p) / (B H W). It equals the L1 loss
    at the base point and is smooth around it; its derivative there is the
    gradient of loss_and_grad (Sec. 4.4 l1 term, decisions held)."""
    B = len(txs)
    H, W = scene.H, scene.W
    count = B * H * W
    pix = M.full_grid(H, W)
    order = M.depth_order(scene.depth)
    xm = M.posenc(M.normalize_mean(scene.mx, scene.my, H, W), M.MEAN_BANDS) if mlp is not None else None
    loss = 0.0
    for b in range(B):
        delta = None
        if mlp is not None:
            xs = M.posenc(M.normalize_tx(txs[b], room), M.TX_BANDS)
            delta, _, _ = M.mlp_forward(xm, xs, mlp, relu_masks=state[b]["masks"])
        g = M.deform(scene, delta)
        rg = M.gaussians_for_raster(g, scene.depth)
        C = M.composite_held(state[b]["rg"], rg, order, pix[0], pix[1])
        t = np.asarray(targets[b], np.float64).ravel()
        loss += float((state[b]["sign"] * (C - t)).sum()) / count
    return loss
