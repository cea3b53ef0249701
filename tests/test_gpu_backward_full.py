"""Gradient parity at the training workload's size: N = 50,000 Gaussians, a
batch of 16 spectra at 90x360, the 4 x 256 network (800k pairs: every
multi-block path of the backward runs as in the training step), BF16 and FP32
forwards and the deterministic BF16 backward, through the C ABI, against the
oracle's FP64 analytic gradient (the
Sec. 3.2 blending rule differentiated with decisions held, through the Sec. 4.1
kernel and the Sec. 4.2 deformation network).

The objective is sum_p w_p C_p with random weights on about 2,000 sampled
pixels per query and zero elsewhere (the oracle composites only those). The
oracle is fed the GPU's own residuals (its compositing layer then sees exactly
the GPU's deformed Gaussians), and sampled pixels where any decision of that
input lies near its threshold are left unweighted, so no decision can differ.

Bounds are componentwise, from the unit roundoffs u32 = 2^-24 and u16 = 2^-8
(8 significant bits) times magnitude sums the oracle accumulates along the same
chain with every factor replaced by its absolute value:
  compositing and covariance part of a Gaussian's gradient:
      (3 m + 32) u32 * base_abs, m the longest composited run at a weighted
      pixel (the replay divides T by (1 - alpha) once per entry and the forward
      multiplied once per entry; 32 covers q, exp and the chain);
  the network's part (weights, biases, the mean features' chain):
      (3 (L + 1) u + L K u32 + 4 sqrt(P) u32 + the compositing bound) * abs,
      u the unit roundoff of the network's operands, L layers of inner width
      K = 256 (FP32 accumulation inside each product), P pairs summed per weight
      (blocked FP32 sums), 3 (L + 1) roundings of operands along the chain (the
      gradient rounded per layer and the upstream gradient once, the forward's
      activations possibly one unit apart from the oracle's emulation).
"""
import math

import numpy as np
import pytest

from oracle import grad as G
from oracle import model as M
from paper_2506_12787_amd import synth
from tests import helpers as Hh

pytestmark = pytest.mark.gpu

N, B, H, W = 50_000, 16, 90, 360
PIX_PER_QUERY = 2000
U32, U16 = 2.0 ** -24, 2.0 ** -8
PARAMS = ("mean_x", "mean_y", "log_scale_x", "log_scale_y", "rotation", "opacity_logit", "amplitude")


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_2506_12787_amd import binding
    assert torch.cuda.is_available(), "GPU test on a machine without a GPU"
    g = synth.gaussians(N, H, W, seed=1002)
    Ws, bs = synth.mlp_weights(seed=3002, out_scale=0.1)
    rng = np.random.default_rng(12)
    bs = [b + rng.normal(0, 0.05, b.shape).astype(np.float32) for b in bs]
    ctx = binding.Context(0)
    sid = ctx.upload_scene(g, H, W, mlp=(Ws, bs))
    tx = torch.from_numpy(synth.tx_positions(B, seed=2002)).cuda()
    yield ctx, sid, M.Scene.from_arrays(g, H, W), Ws, bs, tx
    ctx.release_scene(sid)
    ctx.close()


def _weights(s, deltas, seed):
    """Random weights on sampled pixels whose decisions (for these residuals)
    are all clear of their thresholds."""
    rng = np.random.default_rng(seed)
    order = M.depth_order(s.depth)
    out, kept = [], 0
    for b in range(B):
        idx = rng.choice(H * W, PIX_PER_QUERY, replace=False)
        px, py = (idx % W).astype(np.int32), (idx // W).astype(np.int32)
        rg = M.gaussians_for_raster(M.deform(s, deltas[b]), s.depth)
        res = M.composite(rg, order, px, py)
        ok = idx[res.nflags == 0]
        w = np.zeros(H * W)
        w[ok] = rng.normal(0, 1, len(ok))
        out.append(w)
        kept += len(ok)
    return out, kept


def _compare(name, got, ref, bound):
    got = np.asarray(got, np.float64)
    err = np.abs(got - ref)
    scale = max(float(np.abs(ref).max()), 1e-300)
    ratio = float((err / np.maximum(bound, 1e-300)).max())
    print(f"  {name}: normwise err {err.max() / scale:.2e}, worst err / bound {ratio:.3f}", flush=True)
    return ratio


@pytest.mark.parametrize("mode", ["fp32", "bf16", "bf16-deterministic"])
def test_training_size_gradient_within_derived_bounds(setup, mode):
    # the deterministic backward (fixed-order sums of per-entry partials) is held to the same bounds: it sums the
    # same terms as the atomic one, in another order
    import torch
    from paper_2506_12787_amd import binding as Bd
    ctx, sid, s, Ws, bs, tx = setup
    bf16 = mode.startswith("bf16")
    flags = Bd.MLP_BF16 if bf16 else Bd.MLP_FP32
    bwd_flags = flags | (Bd.DETERMINISTIC if mode.endswith("deterministic") else 0)
    print(f"training-size gradient, {mode}: N={N} B={B}", flush=True)
    deltas = ctx.debug_deform(sid, tx, flags).cpu().numpy().astype(np.float64)
    w, kept = _weights(s, deltas, seed=99 if bf16 else 98)
    print(f"  weighted pixels {kept} of {B * PIX_PER_QUERY} sampled", flush=True)
    out, aux = ctx.render(sid, tx, flags=flags | Bd.KEEP_AUX)
    gr = {k: torch.zeros(N, device="cuda") for k in PARAMS}
    gr["weight"] = [torch.zeros(Wl.shape, device="cuda") for Wl in Ws]
    gr["bias"] = [torch.zeros(Wl.shape[0], device="cuda") for Wl in Ws]
    gw = torch.from_numpy(np.stack(w).astype(np.float32)).cuda()
    ctx.render_backward(sid, tx, bwd_flags, gw, aux, gr)
    torch.cuda.synchronize()
    got = {k: (v.cpu().numpy() if not isinstance(v, list) else [x.cpu().numpy() for x in v]) for k, v in gr.items()}
    mlp = Hh.mlp_f64(Ws, bs)
    txh = tx.cpu().numpy().astype(np.float64)
    _, ref = G.loss_and_grad(s, mlp, txh, None, pixel_weights=w, bf16=bf16, deltas=list(deltas), bounds=True)
    assert not ref["flagged"].any()
    m = ref["replay"]
    L, K, P = len(Ws), 256, B * N
    c_r = (3 * m + 32) * U32
    c_mlp = 3 * (L + 1) * (U16 if bf16 else U32) + L * K * U32 + 4 * math.sqrt(P) * U32 + c_r
    print(f"  longest run {m}: compositing bound factor {c_r:.2e}, network bound factor {c_mlp:.2e}", flush=True)
    worst = {}
    for j, k in enumerate(PARAMS):
        bound = c_r * ref["base_abs"][:, j] + (c_mlp * ref["pe_abs"][:, j] if j < 2 else 0.0)
        worst[k] = _compare(k, got[k], ref["base"][:, j], bound + 1e-300)
    for l in range(L):
        worst[f"W{l}"] = _compare(f"W{l}", got["weight"][l], ref["W"][l], c_mlp * ref["W_abs"][l])
        worst[f"b{l}"] = _compare(f"b{l}", got["bias"][l], ref["b"][l], c_mlp * ref["b_abs"][l])
    bad = {k: v for k, v in worst.items() if not v <= 1.0}
    assert not bad, bad
