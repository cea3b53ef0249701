"""GPU backward pass (blend -> preprocess -> MLP, through the C ABI) against
the oracle's FP64 analytic gradient, for L = sum_p w_p C_p with fixed weights
on the pixels whose decisions are clear of their thresholds, within
componentwise bounds derived from the unit roundoffs (tests/helpers.py:
check_gradients); plus the autograd wrapper, the kept forward state and the
deterministic mode."""
import numpy as np
import pytest

from oracle import grad as G
from oracle import model as M
from paper_2506_12787_amd import synth
from tests import helpers as Hh

pytestmark = pytest.mark.gpu

PARAMS = ("mean_x", "mean_y", "log_scale_x", "log_scale_y", "rotation", "opacity_logit", "amplitude")


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2506_12787_amd import binding
    assert torch.cuda.is_available()
    c = binding.Context(0)
    yield c
    c.close()


def _gpu_grads(ctx, sid, tx, flags, w, n, Ws=None):
    import torch
    from paper_2506_12787_amd import binding as B
    out, aux = ctx.render(sid, tx, flags=flags | B.KEEP_AUX, batch=w.shape[0])
    gr = {k: torch.zeros(n, device="cuda") for k in PARAMS}
    if Ws is not None:
        gr["weight"] = [torch.zeros(W.shape, device="cuda") for W in Ws]
        gr["bias"] = [torch.zeros(W.shape[0], device="cuda") for W in Ws]
    gw = torch.from_numpy(w.astype(np.float32)).cuda()
    ctx.render_backward(sid, tx, flags, gw, aux, gr)
    torch.cuda.synchronize()
    return out, {k: (v.cpu().numpy() if not isinstance(v, list) else [x.cpu().numpy() for x in v])
                 for k, v in gr.items()}


def _gpu_deltas(ctx, sid, tx, flags):
    """The GPU's own residuals (one (n, 7) array per query): the oracle composites exactly the Gaussians the GPU
    deformed, so every decision the weighted pixels depend on is the same on both sides."""
    return list(ctx.debug_deform(sid, tx, flags).cpu().numpy().astype(np.float64))


def _gpu_pattern(ctx, nb, n, layers):
    """The ReLU decisions the last backward used, per query a list of (n, 256) masks (the oracle holds them, as it
    holds the compositing decisions)."""
    if layers == 0:
        return None
    pat = ctx.debug_relu_pattern(nb, n, layers)
    agree = float(pat.mean())
    print(f"  hidden units passing: {agree:.3f}")
    return [[pat[b, :, l, :] for l in range(layers)] for b in range(nb)]


def test_static_backward_matches_fp64(ctx):
    # static scene: compositing and covariance chain only, componentwise within (3 m + 32) u32 of the magnitude
    # sums, every weighted pixel clear of its decision thresholds
    from paper_2506_12787_amd import binding as B
    H, W, n = 90, 360, 300
    g, s = Hh.problem(n, H, W, seed=61)
    sid = ctx.upload_scene(g, H, W)
    w, kept = Hh.unflagged_weights(s, [None], seed=0)
    print(f"  weighted pixels {kept} of {H * W}")
    _, gg = _gpu_grads(ctx, sid, None, B.NO_DEFORM, np.stack(w), n)
    _, ref = G.loss_and_grad(s, None, [None], None, pixel_weights=w, bounds=True)
    Hh.check_gradients(gg, ref, PARAMS, 0, n, bf16=False)
    ctx.release_scene(sid)


@pytest.mark.parametrize("out_scale", [0.1, 1.0])
def test_deformable_fp32_backward_matches_fp64(ctx, out_scale):
    # FP32 network: Gaussians, weights and biases within the derived bounds of the FP32 chain
    import torch
    from paper_2506_12787_amd import binding as B
    H, W, n, nb = 90, 360, 200, 3
    g, s = Hh.problem(n, H, W, seed=71)
    Ws, bs = synth.mlp_weights(seed=3071, out_scale=out_scale)
    rng = np.random.default_rng(5)
    bs = [b + rng.normal(0, 0.05, b.shape).astype(np.float32) for b in bs]
    sid = ctx.upload_scene(g, H, W, mlp=(Ws, bs))
    tx = torch.from_numpy(synth.tx_positions(nb, seed=2071)).cuda()
    deltas = _gpu_deltas(ctx, sid, tx, B.MLP_FP32)
    w, kept = Hh.unflagged_weights(s, deltas, seed=5)
    print(f"  weighted pixels {kept} of {nb * H * W}")
    _, gg = _gpu_grads(ctx, sid, tx, B.MLP_FP32, np.stack(w), n, Ws)
    masks = _gpu_pattern(ctx, nb, n, len(Ws) - 1)
    txh = tx.cpu().numpy().astype(np.float64)
    _, ref = G.loss_and_grad(s, Hh.mlp_f64(Ws, bs), txh, None, pixel_weights=w, deltas=deltas, bounds=True,
                             relu_masks=masks)
    Hh.check_gradients(gg, ref, PARAMS, len(Ws), nb * n, bf16=False)
    ctx.release_scene(sid)


@pytest.mark.parametrize("n_hidden", [4, 2, 1])
def test_deformable_bf16_backward_matches_bf16_oracle(ctx, n_hidden):
    """Backward of a BF16-MLP forward (BF16 activations and GEMM operands, FP32
    accumulation) against the oracle's FP64 gradient of the BF16-rounding
    network, within the derived bounds (u = 2^-8 for the network's operands).
    Depths 4, 2 and 1: with two or more hidden layers the layer-1 gradient is
    formed inside its sums; with one it comes from the output layer and is
    stored in FP32. The distance to the FP64 network's gradient (the BF16
    perturbation of the network itself) is reported."""
    import torch
    from paper_2506_12787_amd import binding as B
    H, W, n, nb = 90, 360, 200, 3
    g, s = Hh.problem(n, H, W, seed=72)
    Ws, bs = synth.mlp_weights(seed=3072, out_scale=0.1, n_hidden=n_hidden)
    rng = np.random.default_rng(6)
    bs = [b + rng.normal(0, 0.05, b.shape).astype(np.float32) for b in bs]
    sid = ctx.upload_scene(g, H, W, mlp=(Ws, bs))
    tx = torch.from_numpy(synth.tx_positions(nb, seed=2072)).cuda()
    deltas = _gpu_deltas(ctx, sid, tx, B.MLP_BF16)
    w, kept = Hh.unflagged_weights(s, deltas, seed=6)
    print(f"  weighted pixels {kept} of {nb * H * W}")
    _, gg = _gpu_grads(ctx, sid, tx, B.MLP_BF16, np.stack(w), n, Ws)
    masks = _gpu_pattern(ctx, nb, n, len(Ws) - 1)
    mlp = Hh.mlp_f64(Ws, bs)
    txh = tx.cpu().numpy().astype(np.float64)
    _, ref = G.loss_and_grad(s, mlp, txh, None, pixel_weights=w, bf16=True, deltas=deltas, bounds=True,
                             relu_masks=masks)
    Hh.check_gradients(gg, ref, PARAMS, len(Ws), nb * n, bf16=True)
    # report: the FP64 network's own gradient (its residuals and activations unrounded)
    _, ref64 = G.loss_and_grad(s, mlp, txh, None, pixel_weights=w)
    for j, k in enumerate(PARAMS):
        e = np.abs(gg[k] - ref64["base"][:, j]).max() / max(np.abs(ref64["base"][:, j]).max(), 1e-300)
        print(f"  {k} against the FP64 network: normwise {e:.2e}")
    for l in range(len(Ws)):
        e = np.abs(gg["weight"][l] - ref64["W"][l]).max() / max(np.abs(ref64["W"][l]).max(), 1e-300)
        print(f"  W{l} against the FP64 network: normwise {e:.2e}")
    ctx.release_scene(sid)


def test_l1_loss_and_gradient(ctx):
    import torch
    rng = np.random.default_rng(3)
    a = rng.normal(0, 1, 100003).astype(np.float32)
    b = rng.normal(0, 1, 100003).astype(np.float32)
    b[:10] = a[:10]
    loss, grad = ctx.l1_loss(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda())
    d = a.astype(np.float64) - b
    assert abs(float(loss.cpu()) - np.abs(d).mean()) <= 1e-6 * np.abs(d).mean()
    np.testing.assert_array_equal(grad.cpu().numpy(), (np.sign(d) / len(a)).astype(np.float32))


def test_autograd_training_step_matches_direct_backward(ctx):
    """torch.autograd through the Renderer module gives the same gradients as
    the direct C-ABI backward, and an Adam step on the L1 loss lowers it."""
    import torch
    from paper_2506_12787_amd import binding as B
    from paper_2506_12787_amd.autograd import Renderer
    H, W, n, nb = 90, 360, 400, 2
    g, s = Hh.problem(n, H, W, seed=81)
    Ws, bs = synth.mlp_weights(seed=3081, out_scale=0.1)
    tx = torch.from_numpy(synth.tx_positions(nb, seed=2081)).cuda()
    gt = M.Scene.from_arrays(synth.gaussians(n, H, W, seed=4081), H, W)
    mlp = Hh.mlp_f64(Ws, bs)
    target = torch.from_numpy(np.stack([M.render_query(gt, mlp, t.astype(np.float64), margins=None)[0].C
                                        .reshape(H, W) for t in tx.cpu().numpy()]).astype(np.float32)).cuda()
    model = Renderer(g, H, W, mlp=(Ws, bs), lib=ctx)
    out = model(tx)
    loss, _ = ctx.l1_loss(out, target)
    lt = (out - target).abs().mean()
    lt.backward()
    auto = [p.grad.clone() for p in model.gauss]
    # direct backward with the L1 upstream gradient sign(out - target) / count
    gw = torch.sign(out.detach() - target) / out.numel()
    _, aux = ctx.render(model.sid, tx, flags=B.KEEP_AUX)
    gd = {k: torch.zeros(n, device="cuda") for k in PARAMS}
    ctx.render_backward(model.sid, tx, 0, gw.contiguous(), aux, gd)
    for a, k in zip(auto, PARAMS):
        np.testing.assert_allclose(a.cpu().numpy(), gd[k].cpu().numpy(), rtol=1e-5, atol=1e-9)
    # one gradient-descent step sized for a 5 % first-order decrease lowers the loss
    params = list(model.parameters())
    for p in params:
        p.grad = None
    l0 = (model(tx) - target).abs().mean()
    l0.backward()
    g2 = sum(float((p.grad ** 2).sum()) for p in params if p.grad is not None)
    eta = 0.05 * float(l0) / g2
    with torch.no_grad():
        for p in params:
            if p.grad is not None:
                p -= eta * p.grad
    l1 = float((model(tx) - target).abs().mean())
    print("L1 before / after one step", float(l0), l1)
    assert l1 < float(l0)
    ctx.release_scene(model.sid)


@pytest.mark.parametrize("bf16", [True, False], ids=["bf16", "fp32"])
def test_backward_takes_the_kept_forward_state(ctx, bf16):
    # right after its forward the backward takes that render's records, lists and (BF16) activations; with another
    # render on the context in between it builds them again: both give the same gradients (up to the order of the
    # blend backward's atomic sums)
    import torch
    from paper_2506_12787_amd import binding as B
    H, W, n, nb = 45, 90, 1500, 3
    g = synth.gaussians(n, H, W, seed=610, scale_range=(1.0, 6.0))
    Ws, bs = synth.mlp_weights(seed=3610, out_scale=0.3)
    sid = ctx.upload_scene(g, H, W, mlp=(Ws, bs))
    tx = torch.from_numpy(synth.tx_positions(nb, seed=710)).cuda()
    flags = B.MLP_BF16 if bf16 else B.MLP_FP32
    w = np.random.default_rng(5).normal(0, 1, (nb, H, W))
    _, g1 = _gpu_grads(ctx, sid, tx, flags, w, n, Ws)
    assert ctx.device_status()["flags"] & B.DEV_BWD_REUSED
    _, aux = ctx.render(sid, tx, flags=flags | B.KEEP_AUX, batch=nb)
    ctx.render(sid, tx[:1].contiguous(), flags=flags)
    gr = {k: torch.zeros(n, device="cuda") for k in PARAMS}
    gr["weight"] = [torch.zeros(x.shape, device="cuda") for x in Ws]
    gr["bias"] = [torch.zeros(x.shape[0], device="cuda") for x in Ws]
    ctx.render_backward(sid, tx, flags, torch.from_numpy(w.astype(np.float32)).cuda(), aux, gr)
    torch.cuda.synchronize()
    assert not ctx.device_status()["flags"] & B.DEV_BWD_REUSED
    for k in PARAMS:
        a, b = g1[k], gr[k].cpu().numpy()
        np.testing.assert_allclose(b, a, rtol=0, atol=1e-5 * np.abs(a).max() + 1e-30, err_msg=k)
    for l, x in enumerate(gr["weight"]):
        a = g1["weight"][l]
        np.testing.assert_allclose(x.cpu().numpy(), a, rtol=0, atol=1e-5 * np.abs(a).max() + 1e-30,
                                   err_msg=f"weight {l}")
    ctx.release_scene(sid)


@pytest.mark.parametrize("bf16", [True, False], ids=["bf16", "fp32"])
def test_deterministic_backward_is_bitwise_repeatable(ctx, bf16):
    # SWF_DETERMINISTIC: per (entry, wave) sums added per pair in the order of its tiles; two backward passes give
    # bitwise the same gradients, which agree with the atomic-add backward to FP32 summation order
    import torch
    from paper_2506_12787_amd import binding as B
    H, W, n, nb = 90, 360, 20_000, 4
    g = synth.gaussians(n, H, W, seed=620, scale_range=(1.0, 8.0))
    Ws, bs = synth.mlp_weights(seed=3620, out_scale=0.3)
    sid = ctx.upload_scene(g, H, W, mlp=(Ws, bs))
    tx = torch.from_numpy(synth.tx_positions(nb, seed=720)).cuda()
    flags = B.MLP_BF16 if bf16 else B.MLP_FP32
    gw = torch.from_numpy(np.random.default_rng(6).normal(0, 1, (nb, H, W)).astype(np.float32)).cuda()
    _, aux = ctx.render(sid, tx, flags=flags | B.KEEP_AUX, batch=nb)

    def run(extra):
        gr = {k: torch.zeros(n, device="cuda") for k in PARAMS}
        gr["weight"] = [torch.zeros(x.shape, device="cuda") for x in Ws]
        gr["bias"] = [torch.zeros(x.shape[0], device="cuda") for x in Ws]
        ctx.render_backward(sid, tx, flags | extra, gw, aux, gr)
        torch.cuda.synchronize()
        return [gr[k] for k in PARAMS] + gr["weight"] + gr["bias"]

    d1 = run(B.DETERMINISTIC)
    d2 = run(B.DETERMINISTIC)
    a1 = run(0)
    a2 = run(0)
    for x, y in zip(d1, d2):
        assert torch.equal(x, y)
    diff_atomic = sum(int(not torch.equal(x, y)) for x, y in zip(a1, a2))
    print(f"atomic-add backward: {diff_atomic} of {len(a1)} gradient blocks differ between two runs", flush=True)
    names = list(PARAMS) + [f"weight {l}" for l in range(len(Ws))] + [f"bias {l}" for l in range(len(Ws))]
    for name, x, y, z in zip(names, d1, a1, a2):
        xs, ys, zs = (t.cpu().numpy().astype(np.float64) for t in (x, y, z))
        scale = np.abs(ys).max() + 1e-30
        e_det, e_atomic = np.abs(xs - ys).max(), np.abs(zs - ys).max()
        print(f"  {name}: deterministic vs atomic {e_det / scale:.1e}, atomic run to run {e_atomic / scale:.1e}")
        # both are the same terms summed in another order: the fixed order is as far from one atomic run as
        # another atomic run is (a few times), plus a floor: FP32 rounding over the blocks' cancelling sums, or,
        # after a BF16 forward, one BF16 unit (2^-8) of the gradients the backward rounds to BF16 (dz of every
        # hidden layer), which a change of summation order can move across a rounding boundary
        floor = 2.0 ** -8 if bf16 else 1e-5
        assert e_det <= 4.0 * e_atomic + floor * scale, name
    ctx.release_scene(sid)
