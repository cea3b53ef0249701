"""Pins of rendering a scene on another resolution of the same field of view
(the render call's grid): at twice the resolution every pixel (2x, 2y) sees
exactly what pixel (x, y) saw at the scene's own grid, for the compositing
model and for the paper's model."""
import numpy as np

from oracle import model as M
from oracle import paper as P
from paper_2506_12787_amd import synth


def test_compositing_model_at_twice_the_resolution():
    H, W = 30, 60
    g = synth.gaussians(300, H, W, seed=240, scale_range=(0.7, 6.0))
    s = M.Scene.from_arrays(g, H, W)
    base, _, _, _ = M.render_query(s, None, None, margins=None)
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    pix = ((2 * xs).ravel().astype(np.int32), (2 * ys).ravel().astype(np.int32))
    two, _, _, _ = M.render_query(s, None, None, margins=None, grid=(2 * H, 2 * W), pix=pix)
    np.testing.assert_allclose(two.C, base.C, rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(two.sig, base.sig)  # the same decisions at every pixel
    # and odd pixels see something else (the grid really is finer)
    odd = ((2 * xs + 1).ravel().astype(np.int32), (2 * ys).ravel().astype(np.int32))
    r_odd, _, _, _ = M.render_query(s, None, None, margins=None, grid=(2 * H, 2 * W), pix=odd)
    assert np.abs(r_odd.C - base.C).max() > 1e-3


def test_paper_model_at_twice_the_resolution():
    H, W = 24, 80
    g = synth.paper_gaussians(200, seed=241, diag=(0.7, 5.0))
    A, _, _, _, _ = P.render_query(g, H, W)
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    pix = ((2 * xs).ravel(), (2 * ys).ravel())
    A2, _, _, _, _ = P.render_query(g, H, W, grid=(2 * H, 2 * W), pix=pix)
    np.testing.assert_allclose(A2, A, rtol=1e-12, atol=1e-14)
