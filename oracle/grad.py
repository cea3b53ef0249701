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


def raster_grad(rg: dict, order, pix, w, flags_out=None, abs_out=None, period: float = 0.0):
    """d(sum_p w_p C_p) / d(mx, my, ixx, ixy, iyy, opacity, amp) per Gaussian.
    flags_out (int8 array of n), if given, receives the near-threshold marks;
    abs_out ((n, 7) float64), if given, the magnitude sums of the terms (the
    scale of a componentwise rounding-error bound, see raster.c)."""
    lib = M._raster()
    n = len(rg["mx"])
    grad = np.zeros((n, 7))
    order = np.ascontiguousarray(order, np.int64)
    px = np.ascontiguousarray(pix[0], np.int32)
    py = np.ascontiguousarray(pix[1], np.int32)
    w = np.ascontiguousarray(w, np.float64)
    consts = np.array([M.ALPHA_MAX, M.ALPHA_MIN, M.T_MIN, M.Q_MAX, float(period)], np.float64)
    P = M._ptr
    marg = np.array(M.DEFAULT_MARGINS, np.float64)
    lib.oracle_grad(n, P(rg["mx"]), P(rg["my"]), P(rg["ixx"]), P(rg["ixy"]), P(rg["iyy"]), P(rg["op"]),
                    P(rg["amp"]), P(rg["live"]), P(order), P(consts), P(marg), len(px), P(px), P(py), P(w), P(grad),
                    None if flags_out is None else P(flags_out), None if abs_out is None else P(abs_out))
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


U32, U16 = 2.0 ** -24, 2.0 ** -8  # unit roundoffs: binary32, bfloat16 (8 significant bits)


def _bf16_gap(v):
    """(distance from v to the nearest boundary of its bfloat16 rounding interval,
    the bfloat16 step at the rounded value); the interval below a power of two is
    half as wide, so there the smaller half-step is taken."""
    r = M.bf16_round(v)
    m, e = np.frexp(r)
    step = np.ldexp(1.0, e - 8)
    half = np.where(np.abs(m) == 0.5, step / 4.0, step / 2.0)
    return half - np.abs(np.asarray(v, np.float64) - r), step


def _decision_slack(x_mean, x_tx, mlp, pres, acts, bf16, relu_masks=None):
    """Per hidden layer: a bound T on |z' - z| between the pre-activation z of
    this network and the z' an implementation in binary32 arithmetic computes
    (FP32 accumulation of K products: (K + 2) u32 times the magnitude sum, plus
    the differences its operands may carry), and a bound on the differences of
    each layer's input operands. Operands: mean and position features computed
    in binary32 (4 u32 of absolute error, |feature| <= 1); with bf16, rounded
    operands agree exactly unless a rounding boundary lies within their slack
    (then they may be one bfloat16 step apart), and a unit whose ReLU decision
    is within its slack may pass up to T. With relu_masks the decisions are
    held: no unit takes the other one, and only the passing units carry slack."""
    rnd = M.bf16_round if bf16 else (lambda a: a)
    dm = x_mean.shape[1]
    W1m, W1s = rnd(mlp.W[0][:, :dm]), mlp.W[0][:, dm:]
    xs = np.atleast_2d(x_tx)
    if bf16:
        gap, step = _bf16_gap(x_mean)
        dxm = np.where(gap <= 4 * U32, step, 0.0)
    else:
        dxm = np.full(x_mean.shape, 4 * U32)
    dxs = np.full(xs.shape[-1], 4 * U32)
    A = np.abs(rnd(x_mean)) @ np.abs(W1m).T + np.abs(xs) @ np.abs(W1s).T + np.abs(mlp.b[0])
    T = [(mlp.W[0].shape[1] + 2) * U32 * A + dxm @ np.abs(W1m).T + np.abs(W1s) @ dxs]
    dins = [np.concatenate([dxm, np.broadcast_to(dxs, (dxm.shape[0], len(dxs)))], -1)]
    for l in range(1, mlp.n_layers):
        z, t, a = pres[l - 1], T[l - 1], acts[l - 1]
        if relu_masks is not None:
            held = relu_masks[l - 1].astype(bool)
            amb = np.zeros(z.shape, bool)
        else:
            held = z > -t
            amb = np.abs(z) <= t
        if bf16:
            gap, step = _bf16_gap(a)
            da = np.where(held & (gap <= t), step, 0.0) + np.where(amb, t * (1.0 + 2.0 ** -7), 0.0)
        else:
            da = np.where(held, t, 0.0)
        dins.append(da)
        if l == mlp.n_layers - 1:
            break
        Wl = np.abs(rnd(mlp.W[l]))
        A = np.abs(rnd(a)) @ Wl.T + np.abs(mlp.b[l])
        T.append((mlp.W[l].shape[1] + 2) * U32 * A + da @ Wl.T)
    return T, dins


def mlp_backward(x_mean, x_tx, mlp: M.MLP, dout, bf16=False, dabs=None, relu_masks=None):
    """Backward of F_theta for rows sharing one TX feature vector. Returns
    (dW list, db list, d x_mean).

    bf16=True differentiates the BF16-rounding network of mlp_forward(bf16=True)
    with its rounded operands (weights, mean features, hidden activations) as
    the operands of every product, arithmetic exact; a rounding has derivative
    one (its operand is treated as the value the forward used). relu_masks
    (one boolean array per hidden layer) holds the activation pattern.

    dabs (magnitudes >= |dout|, same shape), if given, also runs the same chain
    on absolute values, D_L = dabs, D_l = mask_l * (D_{l+1} |W_{l+1}|), and
    returns as a fourth item (A_W, A_b, D_xm): A_W[l] = sum over rows of
    D_l^T |a_{l-1}|, A_b[l] = sum of D_l, D_xm = D_1 |W1m|: the scales of
    componentwise bounds on rounding errors made along the chain. A fifth item
    (F_W, F_b, F_xm) bounds what the decisions of this network's ReLUs may
    change in an implementation that computes the pre-activations in binary32
    (see _decision_slack): a unit whose pre-activation lies within its slack of
    zero may take the other decision, which adds or removes its whole term
    (F_l = amb_l * (D_{l+1} |W_{l+1}|), carried down the chain like D and
    through every unit that may pass it), and operands that may differ by their
    slack add D^T times that slack."""
    out, pres, acts = M.mlp_forward(x_mean, x_tx, mlp, bf16=bf16, relu_masks=relu_masks)
    rnd = M.bf16_round if bf16 else (lambda a: a)
    L = mlp.n_layers
    dW = [None] * L
    db = [None] * L
    AW, Ab = [None] * L, [None] * L
    FW, Fb = [None] * L, [None] * L
    d, D = dout, dabs
    if D is not None:
        T, dins = _decision_slack(x_mean, x_tx, mlp, pres, acts, bf16, relu_masks)
        F = np.zeros_like(D)
    for l in range(L - 1, 0, -1):
        h = rnd(acts[l - 1])
        dW[l] = d.T @ h
        db[l] = d.sum(0)
        Wl = rnd(mlp.W[l])
        mask = (pres[l - 1] > 0) if relu_masks is None else relu_masks[l - 1].astype(bool)
        d = (d @ Wl) * mask
        if D is not None:
            AW[l] = D.T @ np.abs(h)
            Ab[l] = D.sum(0)
            FW[l] = F.T @ np.abs(h) + D.T @ dins[l]
            Fb[l] = F.sum(0)
            G = D @ np.abs(Wl)
            amb = (np.abs(pres[l - 1]) <= T[l - 1]) if relu_masks is None else np.zeros(mask.shape, bool)
            F = (F @ np.abs(Wl)) * (mask | amb) + G * amb
            D = G * mask
    dm = x_mean.shape[1]
    x_full = np.concatenate([rnd(x_mean), np.broadcast_to(np.atleast_2d(x_tx), (x_mean.shape[0], x_tx.shape[-1]))],
                            -1)
    dW[0] = d.T @ x_full
    db[0] = d.sum(0)
    W1m = rnd(mlp.W[0][:, :dm])
    dxm = d @ W1m
    if D is None:
        return dW, db, dxm
    AW[0] = D.T @ np.abs(x_full)
    Ab[0] = D.sum(0)
    FW[0] = F.T @ np.abs(x_full) + D.T @ dins[0]
    Fb[0] = F.sum(0)
    return dW, db, dxm, (AW, Ab, D @ np.abs(W1m)), (FW, Fb, F @ np.abs(W1m))


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


def chain_to_params_abs(g: dict, rg: dict, gabs: np.ndarray) -> np.ndarray:
    """chain_to_params on magnitudes: every linear map of the chain replaced by
    its entrywise absolute value, applied to raster magnitudes gabs (n, 7)."""
    ixx, ixy, iyy = np.abs(rg["ixx"]), np.abs(rg["ixy"]), np.abs(rg["iyy"])
    Ga = np.stack([np.stack([gabs[:, 2], 0.5 * gabs[:, 3]], -1), np.stack([0.5 * gabs[:, 3], gabs[:, 4]], -1)], -2)
    I = np.stack([np.stack([ixx, ixy], -1), np.stack([ixy, iyy], -1)], -2)
    GS = np.einsum("nab,nbc,ncd->nad", I, Ga, I)
    c, s = np.abs(np.cos(g["rot"])), np.abs(np.sin(g["rot"]))
    ex, ey = np.exp(2.0 * g["lsx"]), np.exp(2.0 * g["lsy"])
    dS = {
        "lsx": (2 * c * c * ex, 2 * c * s * ex, 2 * s * s * ex),
        "lsy": (2 * s * s * ey, 2 * c * s * ey, 2 * c * c * ey),
        "rot": (2 * c * s * (ey + ex), (c * c + s * s) * (ex + ey), 2 * c * s * (ex + ey)),
    }
    out = np.zeros((len(c), 7))
    out[:, 0:2] = gabs[:, 0:2]
    for j, k in ((2, "lsx"), (3, "lsy"), (4, "rot")):
        dxx, dxy, dyy = dS[k]
        out[:, j] = GS[:, 0, 0] * dxx + 2.0 * GS[:, 0, 1] * dxy + GS[:, 1, 1] * dyy
    op = g["opacity"]
    out[:, 5] = gabs[:, 5] * op * (1.0 - op)
    out[:, 6] = gabs[:, 6]
    out[~rg["live"].astype(bool)] = 0.0
    return out


def posenc_backward_abs(v, L, dabs):
    """posenc_backward on magnitudes (absolute value of every factor)."""
    v = np.asarray(v, np.float64)
    d = v.shape[-1]
    out = dabs[..., :d].copy()
    for k in range(L):
        f = (2.0 ** k) * np.pi
        out += dabs[..., d * (1 + k): d * (2 + k)] * f * np.abs(np.cos(f * v))
        out += dabs[..., d * (1 + L + k): d * (2 + L + k)] * f * np.abs(np.sin(f * v))
    return out


def loss_and_grad(scene: M.Scene, mlp: M.MLP | None, txs, targets, room=M.DEFAULT_ROOM, stop_grad_pos=False,
                  pixel_weights=None, bf16=False, deltas=None, bounds=False, wrap=False, relu_masks=None):
    """L1 loss over a batch of queries and its FP64 gradient.

    Returns (loss, grads) where grads has 'base' (n, 7) for
    (mx, my, lsx, lsy, rot, logit, amp) and, with an MLP, 'W'/'b' lists.
    With pixel_weights (one array of H*W per query) the objective is instead
    sum_b sum_p w_bp C_bp, and the returned loss is that sum; only the pixels
    with a non-zero weight are composited.

    bf16: the forward and backward of the BF16-rounding network. deltas (one
    (n, 7) array per query, optional): deform with these residuals instead of
    the network's own (e.g. the residuals another implementation computed); the
    MLP backward still uses the network's activations. bounds: grads also holds
    magnitude sums for componentwise error bounds: 'base_abs' (n, 7) of the
    compositing-and-covariance part, 'pe_abs' (n, 2) of the mean features' part
    through the network, 'W_abs' / 'b_abs' of the network's gradients (each the
    absolute-value chain of the same computation), 'replay' = the largest
    number of Gaussians composited at a weighted pixel, and 'W_flip' / 'b_flip'
    / 'pe_flip': what the network's ReLU decisions within binary32 slack of
    zero, and operand differences within that slack, may change (mlp_backward). wrap: periodic azimuth
    (period W, nearest image of each mean). relu_masks (per query, one (n, 256)
    boolean array per hidden layer): the network's activation pattern held at
    the given decisions (e.g. those another implementation took)."""
    B = len(txs)
    H, W = scene.H, scene.W
    count = B * H * W
    pix = M.full_grid(H, W)
    order = M.depth_order(scene.depth)
    gbase = np.zeros((scene.n, 7))
    gflag = np.zeros(scene.n, np.int8)
    gW = [np.zeros_like(w) for w in mlp.W] if mlp is not None else None
    gb = [np.zeros_like(b) for b in mlp.b] if mlp is not None else None
    if bounds:
        base_abs = np.zeros((scene.n, 7))
        pe_abs = np.zeros((scene.n, 2))
        W_abs = [np.zeros_like(w) for w in mlp.W] if mlp is not None else None
        b_abs = [np.zeros_like(b) for b in mlp.b] if mlp is not None else None
        W_flip = [np.zeros_like(w) for w in mlp.W] if mlp is not None else None
        b_flip = [np.zeros_like(b) for b in mlp.b] if mlp is not None else None
        pe_flip = np.zeros((scene.n, 2))
        replay = 0
    loss = 0.0
    period = float(W) if wrap else 0.0
    xm = M.posenc(M.normalize_mean(scene.mx, scene.my, H, W), M.MEAN_BANDS) if mlp is not None else None
    for b in range(B):
        if deltas is not None:
            delta = np.asarray(deltas[b], np.float64)
        else:
            delta = M.deltas(scene, mlp, txs[b], room, bf16=bf16) if mlp is not None else None
        g = M.deform(scene, delta)
        rg = M.gaussians_for_raster(g, scene.depth)
        if pixel_weights is not None:
            w = np.asarray(pixel_weights[b], np.float64).ravel()
            sel = np.nonzero(w)[0]
            res = M.composite(rg, order, pix[0][sel], pix[1][sel], margins=None, period=period)
            loss += float((w[sel] * res.C).sum())
        else:
            res = M.composite(rg, order, pix[0], pix[1], margins=None, period=period)
            t = np.asarray(targets[b], np.float64).ravel()
            loss += np.abs(res.C - t).sum() / count
            w = _pixel_weights(res.C, t, count)
            sel = np.nonzero(w)[0]
        fl = np.zeros(scene.n, np.int8)
        ga = np.zeros((scene.n, 7)) if bounds else None
        gr = raster_grad(rg, order, pix, w, fl, ga, period=period)
        gflag |= fl
        gp = chain_to_params(g, rg, gr)
        gbase += gp
        if bounds:
            gpa = chain_to_params_abs(g, rg, ga)
            base_abs += gpa
            if len(sel):
                replay = max(replay, int(res.ncontrib.max()))
        if mlp is not None:
            xs = M.posenc(M.normalize_tx(txs[b], room), M.TX_BANDS)
            r = mlp_backward(xm, xs, mlp, gp, bf16=bf16, dabs=gpa if bounds else None,
                             relu_masks=None if relu_masks is None else relu_masks[b])
            dW, db, dxm = r[:3]
            for l in range(mlp.n_layers):
                gW[l] += dW[l]
                gb[l] += db[l]
            mu_hat = M.normalize_mean(scene.mx, scene.my, H, W)
            dmu_hat = posenc_backward(mu_hat, M.MEAN_BANDS, dxm)
            gbase[:, 0] += dmu_hat[:, 0] / W
            gbase[:, 1] += dmu_hat[:, 1] / H
            if bounds:
                AW, Ab, Dxm = r[3]
                FW, Fb, Fxm = r[4]
                for l in range(mlp.n_layers):
                    W_abs[l] += AW[l]
                    b_abs[l] += Ab[l]
                    W_flip[l] += FW[l]
                    b_flip[l] += Fb[l]
                pa = posenc_backward_abs(mu_hat, M.MEAN_BANDS, Dxm)
                pe_abs[:, 0] += pa[:, 0] / W
                pe_abs[:, 1] += pa[:, 1] / H
                pf = posenc_backward_abs(mu_hat, M.MEAN_BANDS, Fxm)
                pe_flip[:, 0] += pf[:, 0] / W
                pe_flip[:, 1] += pf[:, 1] / H
    if stop_grad_pos:
        gbase[:, 0:2] = 0.0
    out = dict(base=gbase, W=gW, b=gb, flagged=gflag.astype(bool))
    if bounds:
        out.update(base_abs=base_abs, pe_abs=pe_abs, W_abs=W_abs, b_abs=b_abs, replay=replay, W_flip=W_flip,
                   b_flip=b_flip, pe_flip=pe_flip)
    return loss, out


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
