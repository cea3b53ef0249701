"""The HIP path against the hand-worked examples of tests/golden/ (through
the C ABI): the tile lists, keys and ranges of a six-Gaussian scene bit-exact,
on the binning path and on the full (tile, depth) sort; the composited values
and final transmittances of stacked Gaussians within the FP32 tolerance."""
import numpy as np
import pytest

from tests import helpers as Hh

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2506_12787_amd import binding
    assert torch.cuda.is_available(), "GPU test on a machine without a GPU"
    c = binding.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("full", [False, True])
def test_tile_lists_by_hand(ctx, full):
    from paper_2506_12787_amd import binding as B
    fx = Hh.golden("tile_lists_6g_48x32.json")
    H, W, e = fx["height"], fx["width"], fx["expected"]
    g = Hh.golden_scene(fx)
    sid = ctx.upload_scene(g, H, W)
    ctx.render(sid, None, flags=B.NO_DEFORM | (B.FULL_SORT if full else 0), batch=1)
    dk = ctx.debug_keys(1, len(g["mean_x"]), 6)
    np.testing.assert_array_equal(dk["counts"], e["counts_in_depth_order"])
    np.testing.assert_array_equal(dk["offsets"], e["offsets_in_depth_order"])
    assert len(dk["keys"]) == e["total"]
    keys = [(t << 32) | int(e["depth_bits_hex"][i], 16) for t, i in zip(e["list_tiles"], e["list_ids"])]
    np.testing.assert_array_equal(dk["keys"], np.array(keys, np.uint64))
    np.testing.assert_array_equal(dk["values"], np.array(e["list_ids"], np.uint64))  # query 0
    np.testing.assert_array_equal(dk["ranges"], e["ranges"])
    ctx.release_scene(sid)


@pytest.mark.parametrize("case", range(3))
def test_compositing_by_hand(ctx, case):
    from paper_2506_12787_amd import binding as B
    c = Hh.golden("composite_by_hand.json")["cases"][case]
    sid = ctx.upload_scene(Hh.golden_scene(c), c["height"], c["width"])
    out, aux = ctx.render(sid, None, flags=B.NO_DEFORM | B.KEEP_AUX, batch=1)
    out, T = out[0].cpu().numpy(), aux[0, 0].cpu().numpy()
    want = [Hh.golden_pixel(p) for p in c["pixels"]]
    scale = max(abs(C) for C, _ in want)
    for p, (C, Tw) in zip(c["pixels"], want):
        got_c, got_t = float(out[p["y"], p["x"]]), float(T[p["y"], p["x"]])
        print(c["name"], p["x"], p["y"], got_c, C, got_t, Tw, flush=True)
        assert abs(got_c - C) <= Hh.TOL_REL * scale, (c["name"], p)
        assert abs(got_t - Tw) <= Hh.TOL_REL * max(Tw, 1e-4), (c["name"], p)
    ctx.release_scene(sid)
