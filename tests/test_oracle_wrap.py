"""Pins of the oracle's azimuth wrap (periodic azimuth: 0 and 360 degrees are
one direction, so a Gaussian near the seam also covers the other edge) by
properties independent of its code: a replicated wide plane without wrap, a
cyclic shift, mirror symmetry across the seam, no effect away from it, and
brute-force tile coverage of the folded boxes."""
import numpy as np
import pytest

from oracle import model as M

KEYS = ("mean_x", "mean_y", "log_scale_x", "log_scale_y", "rotation", "opacity_logit", "amplitude", "depth")


def _g(rows):
    a = np.asarray(rows, np.float64)
    return {k: np.ascontiguousarray(a[:, j], np.float32) for j, k in enumerate(KEYS)}


def _seam_scene(W, H, n, seed):
    """Gaussians crowded around the seam (means within 20 px of x = 0 or x = W), on a 2^-10 px lattice so that
    shifts by whole multiples of W stay exact in FP32."""
    rng = np.random.default_rng(seed)
    mx = np.where(rng.uniform(size=n) < 0.5, rng.uniform(0, 20, n), rng.uniform(W - 20, W, n))
    mx = np.round(mx * 1024.0) / 1024.0
    rows = np.stack([mx, rng.uniform(0, H, n), rng.uniform(0, np.log(6), n), rng.uniform(0, np.log(6), n),
                     rng.uniform(0, np.pi, n), rng.normal(0, 1, n), rng.uniform(0, 1, n),
                     rng.uniform(0.5, 10, n)], 1)
    return _g(rows)


def _render(g, H, W, wrap):
    s = M.Scene.from_arrays(g, H, W)
    res, _, _, _ = M.render_query(s, None, None, margins=None, wrap=wrap)
    return res.C.reshape(H, W)


def test_wrap_equals_the_replicated_plane():
    # periodic azimuth on a W-wide grid == the plain plane 3W wide with every Gaussian copied at mx - W, mx, mx + W
    # (copies adjacent in the blending order), seen on its middle third: each pixel there is within the cutoff of at
    # most the copy nearest to it
    H, W, n = 32, 96, 60
    g = _seam_scene(W, H, n, seed=1)
    wrapped = _render(g, H, W, True)
    rep = {k: np.repeat(v, 3) for k, v in g.items()}
    rep["mean_x"] = (np.repeat(g["mean_x"].astype(np.float64), 3) + np.tile([0.0, W, 2.0 * W], n)).astype(np.float32)
    wide = _render(rep, H, 3 * W, False)[:, W:2 * W]
    np.testing.assert_allclose(wrapped, wide, rtol=0, atol=1e-12)
    # and the seam matters here: without wrap the result differs
    assert np.abs(_render(g, H, W, False) - wrapped).max() > 1e-2


def test_cyclic_shift_rotates_the_columns():
    H, W, n, sh = 24, 80, 40, 37
    g = _seam_scene(W, H, n, seed=2)
    base = _render(g, H, W, True)
    g2 = dict(g)
    g2["mean_x"] = (g["mean_x"].astype(np.float64) + sh).astype(np.float32)
    shifted = _render(g2, H, W, True)
    np.testing.assert_allclose(shifted, np.roll(base, sh, axis=1), rtol=0, atol=1e-12)
    # a shift by the full period changes nothing
    g3 = dict(g)
    g3["mean_x"] = (g["mean_x"].astype(np.float64) - W).astype(np.float32)
    np.testing.assert_allclose(_render(g3, H, W, True), base, rtol=0, atol=1e-12)


def test_mirror_symmetry_across_the_seam():
    # an axis-aligned Gaussian centred on column 0: column j equals column W - j
    H, W = 16, 64
    g = _g([[0.0, 8.0, np.log(3.0), np.log(2.0), 0.0, 1.0, 0.8, 1.0]])
    A = _render(g, H, W, True)
    for j in range(1, 12):
        np.testing.assert_allclose(A[:, W - j], A[:, j], rtol=1e-14, atol=0)
    assert A[8, W - 3] > 0.1


def test_no_effect_away_from_the_seam():
    H, W = 32, 128
    g = _g([[64.0, 16.0, np.log(4.0), np.log(3.0), 0.4, 0.5, 0.7, 1.0],
            [40.0, 10.0, np.log(2.0), np.log(5.0), 1.2, -0.3, 0.3, 2.0]])
    np.testing.assert_array_equal(_render(g, H, W, True), _render(g, H, W, False))


@pytest.mark.parametrize("W", [360, 96, 40])
def test_folded_rects_cover_exactly_the_boxes_columns(W):
    # brute force: the columns of a box [x0, x1] taken modulo W, sampled densely (endpoints included)
    H, tile = 16, 16
    TW = -(-W // tile)
    rng = np.random.default_rng(W)
    n = 400
    mx = rng.uniform(-1.5 * W, 2.5 * W, n)
    hx = np.concatenate([rng.uniform(0.2, 0.45 * W, n - 40), rng.uniform(0.45 * W, 0.7 * W, 40)])
    r = M._rect_at(mx, np.full(n, 8.0), hx, np.full(n, 2.0), H, W, tile, wrap=True)
    counts = M.rect_count(r, TW)
    for i in range(n):
        x0, x1 = mx[i] - hx[i], mx[i] + hx[i]
        xs = np.concatenate([np.arange(x0, x1, 0.05), [x1]])
        want = set((np.floor(np.mod(xs, W) / tile)).astype(int).tolist())
        want = {min(c, TW - 1) for c in want}
        tx0, _, tx1, _ = r[i]
        got = set(range(tx0, tx1 + 1)) if tx1 >= tx0 else set(range(tx0, TW)) | set(range(0, tx1 + 1))
        assert got == want, (i, x0, x1, tx0, tx1, sorted(want))
        assert counts[i] == len(got) * (r[i, 3] - r[i, 1] + 1)
