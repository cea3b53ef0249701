"""The paper's own spectrum model (Sec. 4.1 GMM sum over Cholesky Gaussians with
tanh centres and complex responses; Sec. 4.2 / 6.1 deformation MLP with skips)
through the C ABI against the FP64 oracle: spectra within 1e-5 normwise (plus
the bounded contribution of Gaussians whose q lies at the cutoff), the two
channels, the MLP residuals, order independence, culling, and a 64-query launch
at the paper's 10k Gaussians."""
import numpy as np
import pytest

from oracle import paper as P

pytestmark = pytest.mark.gpu
KEYS = ("center_x", "center_y", "chol_l1", "chol_l2", "chol_l3", "atten_logit", "psi_re", "psi_im")
TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    from paper_2506_12787_amd import binding
    c = binding.Context(0)
    yield c
    c.close()


def scene(n, seed, scale=(1.0, 8.0)):
    from paper_2506_12787_amd import synth
    return synth.paper_gaussians(n, seed, diag=scale)


def mlp(seed, out_scale=1.0):
    from paper_2506_12787_amd import synth
    return synth.paper_mlp_weights(seed, out_scale=out_scale)


def check(got, A, bound, tag):
    scale = np.abs(A).max()
    err = np.abs(got.ravel().astype(np.float64) - A)
    ok = err <= TOL * scale + bound
    worst = (err[bound == 0] / scale).max() if (bound == 0).any() else 0.0
    print(f"{tag}: worst unflagged {worst:.2e}, pixels at the cutoff {int((bound > 0).sum())}", flush=True)
    assert ok.all(), (tag, int((~ok).sum()), float(err.max() / scale))


@pytest.mark.parametrize("H,W,n", [(90, 360, 2000), (17, 33, 60), (45, 130, 500), (1, 1, 3)])
def test_static_paper_render(ctx, H, W, n):
    import torch
    from paper_2506_12787_amd import binding as B
    g = scene(n, seed=190 + W)
    sid = ctx.upload_paper_scene(g, H, W)
    out, chan = ctx.render_paper(sid, None, flags=B.NO_DEFORM, batch=2)
    A, re, im, bound = P.render(P.deformed(g, H, W), H, W)
    for q in range(2):
        check(out[q].cpu().numpy(), A, bound, f"static {H}x{W} q{q}")
    c = chan[0].cpu().numpy().reshape(2, -1).astype(np.float64)
    scale = np.abs(A).max()
    assert np.abs(c[0] - re).max() <= TOL * scale + bound.max() and np.abs(c[1] - im).max() <= TOL * scale + bound.max()
    np.testing.assert_allclose(out[0].cpu().numpy().ravel(), np.hypot(c[0], c[1]), rtol=1e-6, atol=1e-7)
    # the sum has no order: the same Gaussians uploaded in another order give the same spectrum (to rounding)
    perm = np.random.default_rng(1).permutation(n)
    sid2 = ctx.upload_paper_scene({k: v[perm] for k, v in g.items()}, H, W)
    out2 = ctx.render(sid2, None, flags=B.NO_DEFORM, batch=1)
    np.testing.assert_allclose(out2[0].cpu().numpy(), out[0].cpu().numpy(), rtol=0, atol=2e-6 * max(scale, 1e-30))
    ctx.release_scene(sid)
    ctx.release_scene(sid2)
    torch.cuda.synchronize()


def test_culled_and_cancelling(ctx):
    from paper_2506_12787_amd import binding as B
    H, W = 32, 64
    g = scene(6, seed=200)
    g["chol_l1"][0] = 0.0          # degenerate: culled
    g["chol_l3"][1] = 0.0
    g["psi_re"][2] = np.nan        # non-finite: culled
    for k in KEYS:                 # Gaussians 4 and 5: identical but opposite responses, so they cancel
        g[k][5] = g[k][4]
    g["psi_re"][5], g["psi_im"][5] = -g["psi_re"][4], -g["psi_im"][4]
    sid = ctx.upload_paper_scene(g, H, W)
    out, _ = ctx.render_paper(sid, None, flags=B.NO_DEFORM, batch=1)
    A, _, _, bound = P.render(P.deformed(g, H, W), H, W)
    check(out[0].cpu().numpy(), A, bound, "culled")
    st = ctx.device_status()
    assert st["culled_nonfinite"] == 3
    ctx.release_scene(sid)


@pytest.mark.parametrize("out_scale", [1.0, 0.1])
def test_deformable_paper_render(ctx, out_scale):
    import torch
    from paper_2506_12787_amd import binding as B
    from paper_2506_12787_amd import synth
    H, W, n, nb = 90, 360, 1500, 3
    g = scene(n, seed=210)
    Ws, bs = mlp(3210, out_scale)
    sid = ctx.upload_paper_scene(g, H, W, mlp=(Ws, bs))
    tx = torch.from_numpy(synth.tx_positions(nb, seed=2210)).cuda()
    out, chan = ctx.render_paper(sid, tx, flags=B.MLP_FP32)
    dd = ctx.debug_deform_paper(sid, tx).cpu().numpy().astype(np.float64)
    txh = tx.cpu().numpy().astype(np.float64)
    moved = 0.0
    for q in range(nb):
        ref = P.mlp_forward(P.features(g, txh[q], H, W), Ws, bs)
        e = np.abs(dd[q] - ref).max() / np.abs(ref).max()
        print(f"paper MLP residuals q{q}: normwise {e:.2e}", flush=True)
        assert e <= 2e-5
        moved = max(moved, np.abs(ref[:, :2]).max())
        A, re, im, bound, _ = P.render_query(g, H, W, mlp=(Ws, bs), tx=txh[q])
        check(out[q].cpu().numpy(), A, bound, f"deformable q{q}")
    print(f"largest centre residual {moved:.2f} px", flush=True)
    ctx.release_scene(sid)


def test_paper_launch_of_64_queries_at_10k(ctx):
    # the paper's Gaussian count, one launch of 64 positions, sampled pixels of 4 queries against the oracle
    import torch
    from paper_2506_12787_amd import binding as B
    from paper_2506_12787_amd import synth
    H, W, n, nb = 90, 360, 10_000, 64
    g = scene(n, seed=220)
    Ws, bs = mlp(3220, 0.3)
    sid = ctx.upload_paper_scene(g, H, W, mlp=(Ws, bs))
    tx = torch.from_numpy(synth.tx_positions(nb, seed=2220)).cuda()
    out, _ = ctx.render_paper(sid, tx, flags=B.MLP_FP32)
    rng = np.random.default_rng(220)
    txh = tx.cpu().numpy().astype(np.float64)
    for q in (0, 21, 42, 63):
        px, py = rng.integers(0, W, 200), rng.integers(0, H, 200)
        A, _, _, bound, _ = P.render_query(g, H, W, mlp=(Ws, bs), tx=txh[q], pix=(px, py))
        got = out[q].cpu().numpy()[py, px]
        # normwise against the full spectrum's scale (the sample's own maximum is a lower bound of it)
        scale = max(np.abs(A).max(), float(out[q].abs().max()))
        err = np.abs(got - A)
        assert (err <= TOL * scale + bound).all(), (q, float(err.max() / scale))
    ctx.release_scene(sid)


def test_invalid_flags(ctx):
    import torch
    from paper_2506_12787_amd import binding as B
    g = scene(10, seed=230)
    sid = ctx.upload_paper_scene(g, 16, 16)
    for f in (B.MLP_BF16, B.NO_DEFORM | B.TILE8, B.NO_DEFORM | B.KEEP_AUX):
        with pytest.raises(B.SwfError):
            ctx.render_paper(sid, torch.zeros((1, 3), device="cuda"), flags=f, batch=1)
    with pytest.raises(B.SwfError):  # no MLP uploaded
        ctx.render_paper(sid, torch.zeros((1, 3), device="cuda"), flags=B.MLP_FP32)
    ctx.release_scene(sid)
