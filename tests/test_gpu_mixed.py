"""Mixed batches (swf_render_mixed): queries over several resident scenes with
different Gaussian counts, grids and MLPs in one launch sequence. Every query
must render bitwise what it renders alone (whose parity with the oracle the
other tests hold), BF16- and FP32-deformed and static; the device status counts
every pair of the batch."""
import numpy as np
import pytest

from oracle import model as M
from paper_2506_12787_amd import synth
from tests import helpers as Hh

pytestmark = pytest.mark.gpu

SCENES = [(5000, 90, 360), (20000, 180, 720), (2000, 45, 130), (700, 16, 16)]


@pytest.fixture(scope="module")
def setup():
    from paper_2506_12787_amd import binding
    ctx = binding.Context(0)
    sids = []
    for i, (n, H, W) in enumerate(SCENES):
        g = synth.gaussians(n, H, W, seed=260 + i)
        sids.append(ctx.upload_scene(g, H, W, mlp=synth.mlp_weights(seed=3260 + i)))
    yield ctx, sids
    ctx.close()


@pytest.mark.parametrize("mode", ["bf16", "fp32", "static"])
def test_mixed_batch_equals_alone(setup, mode):
    import torch
    from paper_2506_12787_amd import binding as B
    ctx, sids = setup
    order = [0, 1, 2, 1, 3, 0, 2, 1, 3, 3, 0]
    ids = [sids[k] for k in order]
    tx = torch.from_numpy(synth.tx_positions(len(ids), seed=2260)).cuda()
    static = mode == "static"
    flags = {"bf16": B.MLP_BF16, "fp32": B.MLP_FP32, "static": B.NO_DEFORM}[mode]
    mixed = ctx.render_mixed(ids, None if static else tx, flags=flags)
    total_pairs = 0
    for b, sid in enumerate(ids):
        alone = ctx.render(sid, None if static else tx[b:b + 1].contiguous(), flags=flags, batch=1)[0]
        assert torch.equal(mixed[b], alone), (b, float((mixed[b] - alone).abs().max()))
        total_pairs += SCENES[order[b]][0]
    ctx.render_mixed(ids, None if static else tx, flags=flags)
    st = ctx.device_status()
    assert st["pairs"] == total_pairs


def test_mixed_batch_against_the_oracle(setup):
    # one query of each scene of a mixed batch, FP64 oracle with the kernel's BF16 rounding
    import torch
    from paper_2506_12787_amd import binding as B
    ctx, sids = setup
    tx = torch.from_numpy(synth.tx_positions(4, seed=2261)).cuda()
    mixed = ctx.render_mixed([sids[2], sids[0], sids[3], sids[2]], tx, flags=B.MLP_BF16)
    for b, k in enumerate([2, 0, 3, 2]):
        n, H, W = SCENES[k]
        g = synth.gaussians(n, H, W, seed=260 + k)
        s = M.Scene.from_arrays(g, H, W)
        Ws, bs = synth.mlp_weights(seed=3260 + k)
        res, _, _, _ = M.render_query(s, Hh.mlp_f64(Ws, bs), tx[b].cpu().numpy().astype(np.float64), bf16=True)
        rep = Hh.parity(mixed[b].cpu().numpy(), res)
        print(f"mixed query {b} (scene {k}): {rep}", flush=True)


def test_mixed_batch_rejects_what_it_does_not_take(setup):
    import torch
    from paper_2506_12787_amd import binding as B
    ctx, sids = setup
    tx = torch.from_numpy(synth.tx_positions(2, seed=2262)).cuda()
    for f in (B.MLP_BF16 | B.KEEP_AUX, B.MLP_BF16 | B.WRAP_AZIMUTH, B.MLP_FP32 | B.TILE8):
        with pytest.raises(B.SwfError):
            ctx.render_mixed([sids[0], sids[1]], tx, flags=f)
    with pytest.raises(B.SwfError):
        ctx.render_mixed([sids[0], 9999], tx, flags=B.MLP_BF16)


def test_mixed_batch_sort_path_for_large_grids(setup):
    # a query grid beyond the binning's tile limit (68 x 68 tiles of 16): the batch takes key emission and the
    # radix sort instead, with the same per-query results
    import torch
    from paper_2506_12787_amd import binding as B
    ctx, sids = setup
    H, W = 1088, 1088
    g = synth.gaussians(3000, H, W, seed=270, scale_range=(2.0, 40.0))
    big = ctx.upload_scene(g, H, W, mlp=synth.mlp_weights(seed=3270))
    ids = [big, sids[2], sids[0], big, sids[3]]
    tx = torch.from_numpy(synth.tx_positions(len(ids), seed=2270)).cuda()
    for flags in (B.MLP_BF16, B.MLP_FP32, B.NO_DEFORM):
        t = None if flags == B.NO_DEFORM else tx
        mixed = ctx.render_mixed(ids, t, flags=flags)
        for b, sid in enumerate(ids):
            alone = ctx.render(sid, None if t is None else tx[b:b + 1].contiguous(), flags=flags, batch=1)[0]
            assert torch.equal(mixed[b], alone), (flags, b)
    ctx.release_scene(big)
