"""Pins of the oracle's analytic L1-loss gradient: central finite differences
with eps = 1e-3 on sampled parameters (with a decision-stability filter), and
closed forms for one Gaussian (Sec. 3.2 blending rule, Sec. 4.1 kernel)."""
import math

import numpy as np
import pytest

from oracle import grad as G
from oracle import model as M
from paper_2506_12787_amd import synth

EPS = 1e-3
RTOL, ATOL = 1e-5, 1e-9
PARAMS = ("mx", "my", "lsx", "lsy", "rot", "logit", "amp")


def _problem(n=200, B=2, H=90, W=360, seed=0, out_scale=0.1, hidden=64):
    g = synth.gaussians(n, H, W, seed=1000 + seed)
    s = M.Scene.from_arrays(g, H, W)
    Ws, bs = synth.mlp_weights(seed=3000 + seed, hidden=hidden, out_scale=out_scale)
    rng = np.random.default_rng(77 + seed)
    mlp = M.MLP([w.astype(np.float64) for w in Ws], [b.astype(np.float64) + rng.normal(0, 0.01, b.shape)
                                                      for b in bs])
    txs = synth.tx_positions(B, seed=2000 + seed).astype(np.float64)
    gt = M.Scene.from_arrays(synth.gaussians(n, H, W, seed=4000 + seed), H, W)
    targets = [M.render_query(gt, mlp, tx, margins=None)[0].C.reshape(H, W) for tx in txs]
    return s, mlp, txs, targets


def _perturb(s, mlp, kind, idx, delta):
    s2 = M.Scene(*(getattr(s, f).copy() if isinstance(getattr(s, f), np.ndarray) else getattr(s, f)
                   for f in ("mx", "my", "lsx", "lsy", "rot", "logit", "amp", "depth", "H", "W")))
    m2 = M.MLP([w.copy() for w in mlp.W], [b.copy() for b in mlp.b])
    if kind in PARAMS:
        getattr(s2, {"logit": "logit", "amp": "amp"}.get(kind, kind))[idx] += delta
    elif kind == "W":
        l, i, j = idx
        m2.W[l][i, j] += delta
    else:
        l, i = idx
        m2.b[l][i] += delta
    return s2, m2


def _samples(mlp, grads, rng):
    """Sample pools: per Gaussian attribute, and the MLP layers interleaved so
    that every layer (weights and a bias) is represented."""
    gb = grads["base"]
    pools = {}
    for j, name in enumerate(PARAMS):
        cand = np.nonzero(np.abs(gb[:, j]) > 1e-9)[0]
        pools[name] = [(name, int(i), gb[i, j]) for i in rng.permutation(cand)]
    mlp_pool = []
    for l in range(mlp.n_layers):
        W = grads["W"][l]
        nz = np.argwhere(np.abs(W) > 1e-9)
        lay = [("W", (l, int(nz[r][0]), int(nz[r][1])), W[nz[r][0], nz[r][1]]) for r in rng.permutation(len(nz))]
        bi = int(np.argmax(np.abs(grads["b"][l])))
        lay.insert(1, ("b", (l, bi), grads["b"][l][bi]))
        mlp_pool.append(lay)
    pools["mlp"] = [x for grp in zip(*[p[:40] for p in mlp_pool]) for x in grp]
    return pools


def test_fd_held_matches_analytic_gradient_training_config():
    # The gradient-check configuration of the training workload: N = 200, a
    # batch of 16 spectra at 90x360, the 4 x 256 network (output scale 0.1 so
    # that the residuals move the Gaussians). At this size almost every eps =
    # 1e-3 perturbation of an MLP weight flips some 3-sigma cutoff somewhere, so
    # instead of rejecting samples the objective is the loss with every discrete
    # decision held at the base point (compositing decisions, ReLU patterns,
    # residual signs): a smooth function equal to the L1 loss at the base point
    # whose derivative is the analytic gradient (decisions held, Sec. 4.4 l1
    # term). 64 parameters: 8 of each Gaussian attribute, 8 MLP weights and
    # biases covering every layer; none is rejected.
    s, mlp, txs, targets = _problem(B=16, hidden=256)
    loss, grads = G.loss_and_grad(s, mlp, txs, targets)
    st = G.held_state(s, mlp, txs, targets)
    assert G.loss_held(s, mlp, txs, targets, st) == pytest.approx(loss, rel=1e-13)
    pools = _samples(mlp, grads, np.random.default_rng(321))
    checked = 0
    for key, pool in pools.items():
        for kind, idx, ana in pool[:8]:
            sp, mp = _perturb(s, mlp, kind, idx, EPS)
            sm, mm = _perturb(s, mlp, kind, idx, -EPS)
            fd = (G.loss_held(sp, mp, txs, targets, st) - G.loss_held(sm, mm, txs, targets, st)) / (2 * EPS)
            assert abs(ana - fd) <= RTOL * abs(fd) + ATOL, (kind, idx, ana, fd)
            checked += 1
    assert checked == 64


def test_fd_matches_analytic_gradient():
    # 64 parameters: 8 of each Gaussian attribute and 8 MLP weights/biases (at
    # least one per layer); a sample whose perturbation changes any decision or
    # residual sign is rejected and redrawn.
    s, mlp, txs, targets = _problem()
    loss, grads = G.loss_and_grad(s, mlp, txs, targets)
    rng = np.random.default_rng(123)
    gb = grads["base"]
    pools = {}
    for j, name in enumerate(PARAMS):
        cand = np.nonzero(np.abs(gb[:, j]) > 1e-9)[0]
        pools[name] = [(name, int(i), gb[i, j]) for i in rng.permutation(cand)]
    mlp_pool = []
    for l in range(mlp.n_layers):
        W = grads["W"][l]
        nz = np.argwhere(np.abs(W) > 1e-9)
        lay = [("W", (l, int(nz[r][0]), int(nz[r][1])), W[nz[r][0], nz[r][1]]) for r in rng.permutation(len(nz))]
        bi = int(np.argmax(np.abs(grads["b"][l])))
        lay.insert(1, ("b", (l, bi), grads["b"][l][bi]))
        mlp_pool.append(lay)
    # interleave layers so that every layer is represented
    pools["mlp"] = [x for grp in zip(*[p[:40] for p in mlp_pool]) for x in grp]
    _, sig0, sgn0 = G.loss_only(s, mlp, txs, targets)
    counts = {}
    for key, pool in pools.items():
        counts[key] = 0
        for kind, idx, ana in pool:
            if counts[key] >= 8:
                break
            sp, mp = _perturb(s, mlp, kind, idx, EPS)
            sm, mm = _perturb(s, mlp, kind, idx, -EPS)
            lp, sigp, sgnp = G.loss_only(sp, mp, txs, targets)
            lm, sigm, sgnm = G.loss_only(sm, mm, txs, targets)
            if not (np.array_equal(sigp, sig0) and np.array_equal(sigm, sig0)
                    and np.array_equal(sgnp, sgn0) and np.array_equal(sgnm, sgn0)):
                continue
            fd = (lp - lm) / (2 * EPS)
            assert abs(ana - fd) <= RTOL * abs(fd) + ATOL, (kind, idx, ana, fd)
            counts[key] += 1
    assert all(c == 8 for c in counts.values()), sorted(counts.items())


def test_single_gaussian_gradient_closed_form():
    # C = amp * o * exp(-q/2) at one pixel: dC/damp = alpha, dC/dmu = amp*alpha*Sigma^-1 d
    H, W = 20, 30
    d = dict(mean_x=[10.3], mean_y=[9.6], log_scale_x=[0.4], log_scale_y=[0.9], rotation=[0.7],
             opacity_logit=[-0.2], amplitude=[0.6], depth=[1.0])
    s = M.Scene.from_arrays(d, H, W)
    gm = M.deform(s, None)
    rg = M.gaussians_for_raster(gm)
    px, py = 11, 8
    w = np.zeros(H * W)
    w[py * W + px] = 1.0
    gr = G.raster_grad(rg, M.depth_order(s.depth), M.full_grid(H, W), w)
    I = np.array([[rg["ixx"][0], rg["ixy"][0]], [rg["ixy"][0], rg["iyy"][0]]])
    dv = np.array([px - gm["mx"][0], py - gm["my"][0]])
    q = dv @ I @ dv
    alpha = gm["opacity"][0] * math.exp(-q / 2)
    assert gr[0, 6] == pytest.approx(alpha, rel=1e-14)
    dmu = gm["amp"][0] * alpha * (I @ dv)
    np.testing.assert_allclose(gr[0, 0:2], dmu, rtol=1e-13)
    assert gr[0, 5] == pytest.approx(gm["amp"][0] * math.exp(-q / 2), rel=1e-14)


def test_magnitude_sums_dominate_the_gradient():
    # The magnitude sums behind the componentwise error bounds are sums of
    # absolute values of the same terms: they dominate the gradient entrywise,
    # and where every term is non-negative (dC/damp = alpha T >= 0 with
    # non-negative pixel weights) they equal it.
    s, mlp, txs, _ = _problem(n=150, B=2)
    rng = np.random.default_rng(4)
    w = [rng.uniform(0, 1, s.H * s.W) * (rng.uniform(0, 1, s.H * s.W) < 0.2) for _ in txs]
    _, ref = G.loss_and_grad(s, mlp, txs, None, pixel_weights=w, bounds=True)
    assert np.all(np.abs(ref["base"][:, 2:]) <= ref["base_abs"][:, 2:] * (1 + 1e-12) + 1e-300)
    np.testing.assert_allclose(ref["base_abs"][:, 6], ref["base"][:, 6], rtol=1e-12, atol=1e-300)
    assert np.all(np.abs(ref["base"][:, :2]) <= (ref["base_abs"][:, :2] + ref["pe_abs"]) * (1 + 1e-12) + 1e-300)
    for l in range(mlp.n_layers):
        assert np.all(np.abs(ref["W"][l]) <= ref["W_abs"][l] * (1 + 1e-12) + 1e-300)
        assert np.all(np.abs(ref["b"][l]) <= ref["b_abs"][l] * (1 + 1e-12) + 1e-300)
    assert ref["replay"] > 0
    # the same with mixed-sign weights: only domination
    w = [rng.normal(0, 1, s.H * s.W) * (rng.uniform(0, 1, s.H * s.W) < 0.2) for _ in txs]
    _, ref = G.loss_and_grad(s, mlp, txs, None, pixel_weights=w, bounds=True)
    assert np.all(np.abs(ref["base"][:, 2:]) <= ref["base_abs"][:, 2:] * (1 + 1e-12) + 1e-300)
    for l in range(mlp.n_layers):
        assert np.all(np.abs(ref["W"][l]) <= ref["W_abs"][l] * (1 + 1e-12) + 1e-300)


def test_residual_override_reproduces_the_network():
    # Feeding the network's own residuals through `deltas` changes nothing (up
    # to the order in which the compositor's threads add their partial sums).
    s, mlp, txs, targets = _problem(n=120, B=2)
    l0, r0 = G.loss_and_grad(s, mlp, txs, targets)
    d = [M.deltas(s, mlp, t) for t in txs]
    l1, r1 = G.loss_and_grad(s, mlp, txs, targets, deltas=d)
    assert l0 == l1
    np.testing.assert_allclose(r0["base"], r1["base"], rtol=1e-12, atol=1e-15 * np.abs(r0["base"]).max())


def _own_pattern(s, mlp, txs):
    xm = M.posenc(M.normalize_mean(s.mx, s.my, s.H, s.W), M.MEAN_BANDS)
    out = []
    for tx in txs:
        xs = M.posenc(M.normalize_tx(tx, M.DEFAULT_ROOM), M.TX_BANDS)
        _, pres, _ = M.mlp_forward(xm, xs, mlp)
        out.append([p > 0 for p in pres])
    return out


def test_held_relu_pattern_of_the_network_itself_changes_nothing():
    # Holding the network's own ReLU decisions reproduces the gradient exactly, and a held pattern can only shrink
    # the allowance for decisions (no unit may take the other one).
    s, mlp, txs, _ = _problem(n=120, B=2)
    rng = np.random.default_rng(8)
    w = [rng.normal(0, 1, s.H * s.W) * (rng.uniform(0, 1, s.H * s.W) < 0.3) for _ in txs]
    _, r0 = G.loss_and_grad(s, mlp, txs, None, pixel_weights=w, bounds=True)
    _, r1 = G.loss_and_grad(s, mlp, txs, None, pixel_weights=w, bounds=True, relu_masks=_own_pattern(s, mlp, txs))
    # (up to the order in which the compositor's threads add their partial sums)
    np.testing.assert_allclose(r1["base"], r0["base"], rtol=1e-12, atol=1e-13 * np.abs(r0["base"]).max())
    for l in range(mlp.n_layers):
        np.testing.assert_allclose(r1["W"][l], r0["W"][l], rtol=1e-12, atol=1e-13 * np.abs(r0["W"][l]).max())
        assert np.all(r1["W_flip"][l] <= r0["W_flip"][l] * (1 + 1e-9) + 1e-15 * r0["W_abs"][l].max())


def test_decision_allowance_covers_a_flipped_unit():
    # A hidden unit whose pre-activation is set within its binary32 slack of zero (by its bias, for one query and
    # Gaussian) may take the other decision: the gradient with that one decision flipped (the pattern held) differs
    # from the network's own by no more than the allowance the oracle gives for its decisions; with the decision
    # held both ways, the allowance has no such term.
    s, mlp, txs, _ = _problem(n=60, B=1, hidden=64)
    xm = M.posenc(M.normalize_mean(s.mx, s.my, s.H, s.W), M.MEAN_BANDS)
    xs = M.posenc(M.normalize_tx(txs[0], M.DEFAULT_ROOM), M.TX_BANDS)
    _, pres, _ = M.mlp_forward(xm, xs, mlp)
    l, k = 1, 5                                   # second hidden layer, unit 5
    p = int(np.argmax(np.abs(pres[l][:, k]) > 0))  # a Gaussian whose unit is not exactly zero
    mlp.b[l][k] -= pres[l][p, k] - 1e-12 * (1.0 + abs(pres[l][p, k]))  # its pre-activation now just above zero
    rng = np.random.default_rng(9)
    w = [rng.normal(0, 1, s.H * s.W)]
    own = _own_pattern(s, mlp, txs)
    assert own[0][l][p, k]
    flipped = [[m.copy() for m in own[0]]]
    flipped[0][l][p, k] = False
    _, r0 = G.loss_and_grad(s, mlp, txs, None, pixel_weights=w, bounds=True)
    _, r1 = G.loss_and_grad(s, mlp, txs, None, pixel_weights=w, bounds=True, relu_masks=flipped)
    moved = 0.0
    for j in range(mlp.n_layers):
        diff = np.abs(r1["W"][j] - r0["W"][j])
        moved = max(moved, float(diff.max()))
        assert np.all(diff <= r0["W_flip"][j] * (1 + 1e-9) + 1e-15 * r0["W_abs"][j].max()), j
        assert np.all(np.abs(r1["b"][j] - r0["b"][j]) <= r0["b_flip"][j] * (1 + 1e-9) + 1e-15 * r0["b_abs"][j].max())
    assert moved > 0.0  # the flip changed the gradient, so the allowance was exercised
    _, r2 = G.loss_and_grad(s, mlp, txs, None, pixel_weights=w, bounds=True, relu_masks=own)
    assert r2["W_flip"][l - 1][k].max() < r0["W_flip"][l - 1][k].max()
