"""Rendering a scene on another resolution of the same field of view
(swf_render_at: e.g. 180 x 720 at 0.5 degree per pixel for a scene uploaded at
90 x 360) against the oracle on that grid: compositing model static and
deformable, the paper's model, integer and non-integer ratios."""
import numpy as np
import pytest

from oracle import model as M
from oracle import paper as P
from paper_2506_12787_amd import synth
from tests import helpers as Hh

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2506_12787_amd import binding
    c = binding.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("grid", [(180, 720), (45, 180), (100, 400), (90, 360)])
def test_static_at_other_resolutions(ctx, grid):
    from paper_2506_12787_amd import binding as B
    H, W = 90, 360
    g, s = Hh.problem(1500, H, W, seed=250)
    sid = ctx.upload_scene(g, H, W)
    out = ctx.render_at(sid, *grid, flags=B.NO_DEFORM).cpu().numpy()
    res, _, _, _ = M.render_query(s, None, None, grid=grid)
    rep = Hh.parity(out[0], res)
    print(f"static at {grid}: {rep}", flush=True)
    if grid == (H, W):
        np.testing.assert_array_equal(out, ctx.render(sid, None, flags=B.NO_DEFORM).cpu().numpy())
    ctx.release_scene(sid)


@pytest.mark.parametrize("mlp", ["fp32", "bf16"])
def test_deformable_at_twice_the_resolution(ctx, mlp):
    import torch
    from paper_2506_12787_amd import binding as B
    H, W, nb = 90, 360, 2
    g, s = Hh.problem(2000, H, W, seed=251)
    bf16 = mlp == "bf16"
    Ws, bs = synth.mlp_weights(seed=3251, out_scale=0.01 if bf16 else 1.0)
    sid = ctx.upload_scene(g, H, W, mlp=(Ws, bs))
    tx = torch.from_numpy(synth.tx_positions(nb, seed=2251)).cuda()
    out = ctx.render_at(sid, 180, 720, tx, flags=B.MLP_BF16 if bf16 else B.MLP_FP32).cpu().numpy()
    m64 = Hh.mlp_f64(Ws, bs)
    for q, t in enumerate(tx.cpu().numpy().astype(np.float64)):
        res, _, _, _ = M.render_query(s, m64, t, bf16=bf16, grid=(180, 720))
        rep = Hh.parity(out[q], res)
        print(f"deformable {mlp} at 180x720 q{q}: {rep}", flush=True)
    with pytest.raises(B.SwfError):  # the backward's aux needs the scene's own grid
        ctx._check(ctx._L.swf_render_at(ctx._h, sid, tx.data_ptr(), nb, 180, 720, B.MLP_FP32 | B.KEEP_AUX,
                                        torch.empty((nb, 180, 720), device="cuda").data_ptr(),
                                        torch.empty((2, nb, 180, 720), device="cuda").data_ptr(), None))
    ctx.release_scene(sid)


def test_paper_model_at_twice_the_resolution(ctx):
    import torch
    from paper_2506_12787_amd import binding as B
    H, W, nb = 90, 360, 2
    g = synth.paper_gaussians(1500, seed=252)
    Ws, bs = synth.paper_mlp_weights(seed=3252, out_scale=0.3)
    sid = ctx.upload_paper_scene(g, H, W, mlp=(Ws, bs))
    tx = torch.from_numpy(synth.tx_positions(nb, seed=2252)).cuda()
    out = ctx.render_at(sid, 180, 720, tx, flags=B.MLP_FP32).cpu().numpy()
    for q, t in enumerate(tx.cpu().numpy().astype(np.float64)):
        A, _, _, bound, _ = P.render_query(g, H, W, mlp=(Ws, bs), tx=t, grid=(180, 720))
        scale = np.abs(A).max()
        err = np.abs(out[q].ravel().astype(np.float64) - A)
        assert (err <= 1e-5 * scale + bound).all(), (q, float(err.max() / scale))
    ctx.release_scene(sid)
