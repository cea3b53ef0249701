"""Pins of the oracle's tile binning, key construction and scan (the tile
partitioning of Sec. 4.1) against brute force on small inputs."""
import numpy as np

from oracle import model as M
from paper_2506_12787_amd import synth


def test_depth_bits_preserve_float_order():
    rng = np.random.default_rng(1)
    d = np.concatenate([rng.normal(0, 5, 5000), [0.0, -0.0, 1e-30, -1e-30, 1e30, -1e30]]).astype(np.float32)
    bits = M.depth_bits(d)
    for i in range(0, len(d) - 1):
        a, b = d[i], d[i + 1]
        assert (a < b) == (bits[i] < bits[i + 1])
        assert (a == b) == (bits[i] == bits[i + 1])
    assert M.depth_bits(np.array([-0.0], np.float32))[0] == M.depth_bits(np.array([0.0], np.float32))[0]


def _scene(n, H, W, seed):
    g = synth.gaussians(n, H, W, seed=seed)
    s = M.Scene.from_arrays(g, H, W)
    gm = M.deform(s, None)
    return s, gm, M.gaussians_for_raster(gm)


def test_rect_contains_every_pixel_inside_the_cutoff():
    H, W, tile = 50, 90, 16
    s, gm, rg = _scene(400, H, W, seed=2)
    rect, flagged, _ = M.tile_rects(gm, rg, H, W, tile)
    xs, ys = M.full_grid(H, W)
    for i in range(s.n):
        d = np.stack([xs - gm["mx"][i], ys - gm["my"][i]], -1)
        I = np.array([[rg["ixx"][i], rg["ixy"][i]], [rg["ixy"][i], rg["iyy"][i]]])
        q = np.einsum("pa,ab,pb->p", d, I, d)
        inside = q <= 9.0
        if not inside.any():
            continue
        assert rect[i, 0] >= 0
        tx, ty = xs[inside] // tile, ys[inside] // tile
        assert tx.min() >= rect[i, 0] and tx.max() <= rect[i, 2]
        assert ty.min() >= rect[i, 1] and ty.max() <= rect[i, 3]


def test_rect_tiles_all_touch_the_extent_box():
    H, W, tile = 50, 90, 8
    s, gm, rg = _scene(300, H, W, seed=3)
    rect, _, _ = M.tile_rects(gm, rg, H, W, tile)
    hx = 3 * np.sqrt(rg["sxx"]) + M.EXTENT_EPS
    hy = 3 * np.sqrt(rg["syy"]) + M.EXTENT_EPS
    for i in range(s.n):
        if rect[i, 0] < 0:
            box_hits = (gm["mx"][i] + hx[i] >= 0) and (gm["mx"][i] - hx[i] <= W - 1) and \
                       (gm["my"][i] + hy[i] >= 0) and (gm["my"][i] - hy[i] <= H - 1)
            assert not box_hits
            continue
        # first and last tile column overlap [mx - hx, mx + hx] clipped to the grid
        assert rect[i, 0] * tile <= max(gm["mx"][i] + hx[i], 0)
        assert (rect[i, 2] + 1) * tile > min(gm["mx"][i] - hx[i], W - 1)
        assert rect[i, 1] * tile <= max(gm["my"][i] + hy[i], 0)
        assert (rect[i, 3] + 1) * tile > min(gm["my"][i] - hy[i], H - 1)


def test_key_list_matches_brute_force_per_tile():
    H, W, tile = 40, 70, 16
    s, gm, rg = _scene(150, H, W, seed=4)
    rect, _, _ = M.tile_rects(gm, rg, H, W, tile)
    gt, dk, ids, ranges = M.key_list(rect, s.depth, H, W, tile)
    TW, TH = -(-W // tile), -(-H // tile)
    for t in range(TW * TH):
        tx, ty = t % TW, t // TW
        members = [i for i in range(s.n) if rect[i, 0] >= 0 and rect[i, 0] <= tx <= rect[i, 2]
                   and rect[i, 1] <= ty <= rect[i, 3]]
        members.sort(key=lambda i: (float(np.float32(s.depth[i])), i))
        a, b = ranges[t]
        assert list(ids[a:b]) == members
        assert np.all(gt[a:b] == t)
    assert ranges[-1, 1] == len(gt)


def test_flagged_rect_lists_both_tilings():
    H, W, tile = 40, 70, 16
    # isotropic sigma 1 (h = 3.001) with mx - h landing on the tile edge x = 16
    d = dict(mean_x=[16.0 + 3.0 + float(np.float32(1e-3))], mean_y=[20.0], log_scale_x=[0.0], log_scale_y=[0.0],
             rotation=[0.0], opacity_logit=[0.0], amplitude=[1.0], depth=[1.0])
    s = M.Scene.from_arrays(d, H, W)
    gm = M.deform(s, None)
    rg = M.gaussians_for_raster(gm)
    rect, flagged, alts = M.tile_rects(gm, rg, H, W, tile)
    assert flagged[0]
    assert {a[0] for a in alts[0]} == {0, 1}


def test_exclusive_scan():
    off, tot = M.exclusive_scan(np.ones(10, np.uint32))
    assert list(off) == list(range(10)) and tot == 10
    c = np.random.default_rng(0).integers(0, 100, 1000)
    off, tot = M.exclusive_scan(c)
    assert off[0] == 0 and tot == c.sum()
    assert np.all(np.diff(off.astype(np.int64)) == c[:-1])
    off, tot = M.exclusive_scan(np.full(3, 2 ** 31, np.uint64))
    assert tot == 3 * 2 ** 31
