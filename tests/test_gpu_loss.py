"""Hybrid training loss (paper Sec. 4.4: lambda1 * l1 + (1 - lambda1) * (1 - SSIM))
through the C ABI against the FP64 oracle: loss values and the gradient with
respect to the prediction, on ragged and full-size spectra, plus edge cases
(identical images, lambda1 = 1 is the l1 loss, 1 x 1 images)."""
import numpy as np
import pytest

from oracle import ssim as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2506_12787_amd import binding
    c = binding.Context(0)
    yield c
    c.close()


def _run(ctx, p, t, lam):
    import torch
    pd = torch.from_numpy(p.astype(np.float32)).cuda()
    td = torch.from_numpy(t.astype(np.float32)).cuda()
    loss, grad = ctx.hybrid_loss(pd, td, lam)
    return loss.cpu().numpy().astype(np.float64), grad.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("B,H,W", [(2, 90, 360), (3, 17, 33), (1, 45, 130), (16, 16, 16), (2, 1, 1), (1, 5, 200)])
@pytest.mark.parametrize("lam", [0.7, 0.0])
def test_hybrid_loss_matches_oracle(ctx, B, H, W, lam):
    rng = np.random.default_rng(B * 1000 + H + W)
    t = rng.uniform(0, 1, (B, H, W)).astype(np.float32)
    # a prediction near the target (the training regime) with some smooth structure
    p = np.clip(t + rng.normal(0, 0.1, t.shape), 0, 1.2).astype(np.float32)
    loss, grad = _run(ctx, p, t, lam)
    ref, l1, ssim, gref = S.hybrid_loss_and_grad(p.astype(np.float64), t.astype(np.float64), lam)
    assert loss[1] == pytest.approx(l1, rel=1e-6)
    assert loss[2] == pytest.approx(ssim, rel=1e-6, abs=1e-7)
    assert loss[0] == pytest.approx(ref, rel=1e-6, abs=1e-7)
    err = np.abs(grad - gref).max() / np.abs(gref).max()
    print(f"B={B} {H}x{W} lambda1={lam}: loss {loss[0]:.6f} vs {ref:.6f}, gradient normwise {err:.2e}")
    assert err <= 1e-5


def test_identical_images_and_pure_l1(ctx):
    rng = np.random.default_rng(7)
    t = rng.uniform(0, 1, (3, 40, 70)).astype(np.float32)
    loss, grad = _run(ctx, t, t, 0.7)
    assert loss[2] == pytest.approx(1.0, abs=1e-7) and abs(loss[0]) <= 1e-7 and loss[1] == 0.0
    assert np.abs(grad).max() <= 1e-9
    p = (t + 0.05).astype(np.float32)
    loss, grad = _run(ctx, p, t, 1.0)
    assert loss[0] == pytest.approx(np.abs(p.astype(np.float64) - t).mean(), rel=1e-6)
    np.testing.assert_allclose(grad, np.sign(p.astype(np.float64) - t) / p.size, rtol=1e-6)


def test_invalid_arguments(ctx):
    import torch
    from paper_2506_12787_amd import binding as B
    x = torch.zeros((1, 8, 8), device="cuda")
    with pytest.raises(B.SwfError):
        ctx.hybrid_loss(x, x, 1.5)
    with pytest.raises(B.SwfError):
        ctx.hybrid_loss(x, x, -0.1)
