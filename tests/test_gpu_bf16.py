"""BF16-MFMA deformation MLP: exact fragment-layout pin, error report against
the FP32 GPU path and the FP64 oracle, and render parity against the oracle
running the same BF16 operand rounding."""
import numpy as np
import pytest

from oracle import model as M
from paper_2506_12787_amd import synth
from tests import helpers as Hh

pytestmark = pytest.mark.gpu

H0, W0 = 90, 360


@pytest.fixture(scope="module", params=[0, 32, 64], ids=["ppw48", "ppw32", "ppw64"])
def ctx(request):
    """The three register-tile variants of the MFMA kernel: 48 pairs per wave
    (the default; 384-pair workgroups), 32 and 64 (256-pair workgroups)."""
    import torch
    from paper_2506_12787_amd import binding
    assert torch.cuda.is_available()
    c = binding.Context(0, mlp_pairs_per_wave=request.param)
    yield c
    c.close()


def _exact_mlp(seed):
    """Sparse dyadic weights: every operand, partial sum and activation is
    exactly representable in bfloat16, so any fragment-layout mistake shows as
    a bit difference."""
    rng = np.random.default_rng(seed)
    W1 = np.zeros((256, 89), np.float32)
    for r in range(256):
        W1[r, rng.choice(26, 2, replace=False)] = rng.choice([0.5, 1.0], 2)
    b1 = (rng.integers(-2, 3, 256) * 0.25).astype(np.float32)
    Ws, bs = [W1], [b1]
    for _ in range(3):
        W = np.zeros((256, 256), np.float32)
        for r in range(256):
            W[r, rng.choice(256, 2, replace=False)] = 0.5
        Ws.append(W)
        bs.append(np.zeros(256, np.float32))
    Wo = np.zeros((7, 256), np.float32)
    for r in range(7):
        Wo[r, rng.choice(256, 2, replace=False)] = rng.choice([0.5, -0.5], 2)
    Ws.append(Wo)
    bs.append((rng.integers(-2, 3, 7) * 0.125).astype(np.float32))
    return Ws, bs


@pytest.mark.parametrize("n", [37, 300, 1000])
def test_mfma_fragment_layout_bit_exact(ctx, n):
    import torch
    from paper_2506_12787_amd import binding as B
    rng = np.random.default_rng(n)
    g = synth.gaussians(n, H0, W0, seed=n)
    g["mean_x"] = rng.choice([0.0, W0 / 2], n).astype(np.float32)
    g["mean_y"] = rng.choice([0.0, H0 / 2], n).astype(np.float32)
    Ws, bs = _exact_mlp(n)
    sid = ctx.upload_scene(g, H0, W0, mlp=(Ws, bs))
    tx = torch.from_numpy(synth.tx_positions(3, seed=n + 1)).cuda()
    d16 = ctx.debug_deform(sid, tx, flags=B.MLP_BF16).cpu().numpy().astype(np.float64)
    d32 = ctx.debug_deform(sid, tx, flags=B.MLP_FP32).cpu().numpy().astype(np.float64)
    s = M.Scene.from_arrays(g, H0, W0)
    mlp = Hh.mlp_f64(Ws, bs)
    for b in range(3):
        ref = M.deltas(s, mlp, tx[b].cpu().numpy().astype(np.float64), bf16=True)
        assert np.abs(ref).max() > 0
        np.testing.assert_array_equal(d16[b], ref)
        np.testing.assert_array_equal(d32[b], ref)
    ctx.release_scene(sid)


@pytest.mark.parametrize("out_scale", [0.01, 1.0])
def test_bf16_residual_error_report(ctx, out_scale):
    """Reported, not gated against FP64: BF16 residuals vs FP32 GPU and FP64.
    Gated against the oracle with the same BF16 operand rounding."""
    import torch
    from paper_2506_12787_amd import binding as B
    n, nb = 20000, 4
    g, s = Hh.problem(n, H0, W0, seed=1001)
    Ws, bs = synth.mlp_weights(seed=3001, out_scale=out_scale)
    sid = ctx.upload_scene(g, H0, W0, mlp=(Ws, bs))
    tx = torch.from_numpy(synth.tx_positions(nb, seed=2001)).cuda()
    d16 = ctx.debug_deform(sid, tx, flags=B.MLP_BF16).cpu().numpy().astype(np.float64)
    d32 = ctx.debug_deform(sid, tx, flags=B.MLP_FP32).cpu().numpy().astype(np.float64)
    mlp = Hh.mlp_f64(Ws, bs)
    rep = {"vs_fp32": 0.0, "vs_fp64": 0.0, "vs_bf16_oracle": 0.0}
    for b in range(nb):
        txh = tx[b].cpu().numpy().astype(np.float64)
        r64 = M.deltas(s, mlp, txh)
        r16 = M.deltas(s, mlp, txh, bf16=True)
        scale = np.abs(r64).max(axis=0)
        rep["vs_fp32"] = max(rep["vs_fp32"], float((np.abs(d16[b] - d32[b]).max(0) / scale).max()))
        rep["vs_fp64"] = max(rep["vs_fp64"], float((np.abs(d16[b] - r64).max(0) / scale).max()))
        rep["vs_bf16_oracle"] = max(rep["vs_bf16_oracle"], float((np.abs(d16[b] - r16).max(0) / scale).max()))
    print("BF16 residual normwise relative error", out_scale, rep)
    # FP32 accumulation order vs FP64 flips the BF16 re-rounding of some hidden
    # activations by one ulp (2^-8 relative); those flips propagate, so the
    # kernel sits ~1e-2 from the BF16-emulating oracle and closer to it than to
    # the FP64 MLP.
    assert rep["vs_bf16_oracle"] < 2e-2
    assert rep["vs_bf16_oracle"] < rep["vs_fp64"]
    assert rep["vs_fp64"] < 5e-2
    ctx.release_scene(sid)


def test_bf16_render_parity_with_bf16_oracle(ctx):
    import torch
    from paper_2506_12787_amd import binding as B
    n, nb = 5000, 3
    g, s = Hh.problem(n, H0, W0, seed=1007)
    Ws, bs = synth.mlp_weights(seed=3007)
    sid = ctx.upload_scene(g, H0, W0, mlp=(Ws, bs))
    tx = torch.from_numpy(synth.tx_positions(nb, seed=2007)).cuda()
    out16 = ctx.render(sid, tx, flags=B.MLP_BF16).cpu().numpy()
    out32 = ctx.render(sid, tx, flags=B.MLP_FP32).cpu().numpy()
    mlp = Hh.mlp_f64(Ws, bs)
    for b in range(nb):
        txh = tx[b].cpu().numpy().astype(np.float64)
        res16, _, _, _ = M.render_query(s, mlp, txh, bf16=True)
        rep = Hh.parity(out16[b], res16)
        res64, _, _, _ = M.render_query(s, mlp, txh, margins=None)
        e64 = float(np.abs(out16[b].ravel() - res64.C).max() / np.abs(res64.C).max())
        e32 = float(np.abs(out16[b] - out32[b]).max() / np.abs(out32[b]).max())
        print("BF16 render: parity vs BF16 oracle", rep, "| normwise vs FP64 oracle", e64, "vs FP32 GPU", e32)
    ctx.release_scene(sid)


def test_device_side_mlp_update_matches_upload(ctx):
    """An MLP update from device tensors rebuilds the BF16 weight stream and the
    FP32 fragment-major copy on the device. Renders after it (BF16 and FP32 MLP)
    are bitwise those of the same weights uploaded from the host (the BF16
    stream packed on the host there); a scene updated to other weights and back
    gives the original renders again."""
    import torch
    from paper_2506_12787_amd import binding as B
    g, s = Hh.problem(3000, H0, W0, seed=77)
    Ws, bs = synth.mlp_weights(seed=78, out_scale=1.0)
    W2, b2 = synth.mlp_weights(seed=79, out_scale=1.0)
    tx = torch.from_numpy(synth.tx_positions(3, seed=80)).cuda()
    ref = ctx.upload_scene(g, H0, W0, mlp=(Ws, bs))
    want = {f: ctx.render(ref, tx, flags=f).cpu() for f in (B.MLP_BF16, B.MLP_FP32)}
    sid = ctx.upload_scene(g, H0, W0, mlp=(W2, b2))
    other = ctx.render(sid, tx, flags=B.MLP_BF16).cpu()
    assert not torch.equal(other, want[B.MLP_BF16])
    dev = lambda a: [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in a]
    ctx.update_scene(sid, mlp=(dev(Ws), dev(bs)))
    for f, w in want.items():
        assert torch.equal(ctx.render(sid, tx, flags=f).cpu(), w), f
    ctx.release_scene(sid)
    ctx.release_scene(ref)
