"""Pins of the oracle against worked examples derived by hand (tests/golden/):
tile lists and keys (Sec. 4.1 tile partitioning), front-to-back compositing
(Sec. 3.2) with the kernel weight of Sec. 4.1, and the positional encoding of
Sec. 4.2. The paper prints no worked example; each fixture states its own
derivation, and its expected values are integers or closed forms."""
import numpy as np
import pytest

from oracle import model as M
from tests import helpers as Hh


def test_tile_lists_by_hand():
    fx = Hh.golden("tile_lists_6g_48x32.json")
    H, W, e = fx["height"], fx["width"], fx["expected"]
    s = M.Scene.from_arrays(Hh.golden_scene(fx), H, W)
    gm = M.deform(s, None)
    rg = M.gaussians_for_raster(gm, s.depth)
    rect, flagged, _ = M.tile_rects(gm, rg, H, W, 16)
    assert not flagged.any()
    np.testing.assert_array_equal(rect, e["rects_tx0_ty0_tx1_ty1"])
    order = M.depth_order(s.depth)
    np.testing.assert_array_equal(order, e["depth_order"])
    counts = M.rect_count(rect)[order]
    np.testing.assert_array_equal(counts, e["counts_in_depth_order"])
    offs, tot = M.exclusive_scan(counts)
    np.testing.assert_array_equal(offs, e["offsets_in_depth_order"])
    assert tot == e["total"]
    np.testing.assert_array_equal(M.depth_bits(s.depth), [int(h, 16) for h in e["depth_bits_hex"]])
    gt, dk, ids, ranges = M.key_list(rect, s.depth, H, W)
    np.testing.assert_array_equal(gt, e["list_tiles"])
    np.testing.assert_array_equal(ids, e["list_ids"])
    np.testing.assert_array_equal(dk, [int(e["depth_bits_hex"][i], 16) for i in e["list_ids"]])
    np.testing.assert_array_equal(ranges, e["ranges"])


@pytest.mark.parametrize("case", range(3))
def test_compositing_by_hand(case):
    c = Hh.golden("composite_by_hand.json")["cases"][case]
    s = M.Scene.from_arrays(Hh.golden_scene(c), c["height"], c["width"])
    px = np.array([p["x"] for p in c["pixels"]], np.int32)
    py = np.array([p["y"] for p in c["pixels"]], np.int32)
    res, _, _, _ = M.render_query(s, None, None, pix=(px, py))
    for i, p in enumerate(c["pixels"]):
        C, T = Hh.golden_pixel(p)
        assert res.C[i] == pytest.approx(C, rel=1e-14, abs=1e-300), (c["name"], p)
        assert res.T[i] == pytest.approx(T, rel=1e-14, abs=1e-300), (c["name"], p)
        if "n_contrib" in p:
            assert res.ncontrib[i] == p["n_contrib"]


@pytest.mark.parametrize("case", range(3))
def test_posenc_by_hand(case):
    c = Hh.golden("posenc_by_hand.json")["cases"][case]
    if c["kind"] == "tx":
        p = M.normalize_tx(np.array(c["input"]))
    else:
        p = M.normalize_mean(np.array([c["input"][0]]), np.array([c["input"][1]]), c["height"], c["width"])[0]
    g = M.posenc(p, c["bands"])
    f = lambda rows: [Hh.closed_form(x) for r in rows for x in r]
    expect = [Hh.closed_form(x) for x in c["p"]] + f(c["sin"]) + f(c["cos"])
    assert len(g) == len(expect) == len(p) * (2 * c["bands"] + 1)
    # sin and cos of 2^k pi p are exact up to the rounding of their argument in
    # float64: allow a few units in the last place of the argument
    arg = np.r_[np.zeros(len(p)), np.tile(np.outer(2.0 ** np.arange(c["bands"]), np.pi * p).ravel(), 2)]
    assert np.all(np.abs(g - expect) <= 4 * np.finfo(np.float64).eps * (1 + np.abs(arg)))
