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


def _mlp_fixture():
    from fractions import Fraction
    fx = Hh.golden("mlp_bf16_by_hand.json")
    fr = lambda s: float(Fraction(s))
    xm = np.zeros((1, 26))
    for k, v in fx["x_mean"].items():
        xm[0, int(k)] = fr(v)
    xs = np.zeros(63)
    for k, v in fx["x_tx"].items():
        xs[int(k)] = fr(v)
    Ws, bs = [], []
    for lay in fx["layers"]:
        w = np.zeros((lay["out"], lay["in"]))
        for k, v in lay["weight"].items():
            i, j = (int(t) for t in k.split(","))
            w[i, j] = fr(v)
        Ws.append(w)
        bs.append(np.array([fr(v) for v in lay["bias"]]))
    return fx, xm, xs, M.MLP(Ws, bs), fr


def test_bf16_mlp_emulation_by_hand():
    # Every rounding point of the BF16 emulation (mean features, weights,
    # hidden activations, ties to even) and the unrounded transceiver term and
    # biases change an expected value of the hand-derived network.
    fx, xm, xs, mlp, fr = _mlp_fixture()
    out, pres, _ = M.mlp_forward(xm, xs, mlp, bf16=True)
    e = fx["expected_bf16"]
    for l in range(2):
        np.testing.assert_array_equal(pres[l][0], [fr(v) for v in e["pre"][l]])
    np.testing.assert_array_equal(out[0], [fr(v) for v in e["out"]])
    out, pres, _ = M.mlp_forward(xm, xs, mlp, bf16=False)
    e = fx["expected_fp64"]
    for l in range(2):
        np.testing.assert_allclose(pres[l][0], [fr(v) for v in e["pre"][l]], rtol=2e-16, atol=0)
    np.testing.assert_allclose(out[0], [fr(v) for v in e["out"]], rtol=2e-16, atol=0)


def test_bf16_mlp_fixture_detects_planted_rounding_mistakes(monkeypatch):
    # The fixture must fail an emulation that rounds ties away from zero or one
    # that skips rounding altogether.
    fx, xm, xs, mlp, fr = _mlp_fixture()
    want = [fr(v) for v in fx["expected_bf16"]["pre"][0]] + [fr(v) for v in fx["expected_bf16"]["out"]]

    def ties_away(x):
        x = np.asarray(x, np.float64)
        m, ex = np.frexp(x)
        return np.ldexp(np.sign(m) * np.floor(np.abs(m) * 256.0 + 0.5) / 256.0, ex)

    for wrong in (ties_away, lambda x: np.asarray(x, np.float64)):
        monkeypatch.setattr(M, "bf16_round", wrong)
        out, pres, _ = M.mlp_forward(xm, xs, mlp, bf16=True)
        assert not np.array_equal(np.concatenate([pres[0][0], out[0]]), want)


def test_bf16_mlp_backward_by_hand():
    # Upstream gradient 1 on output 0 of the hand network. Through the
    # BF16-rounding network each product uses the forward's rounded operands:
    # d out0 / d pre1 = (bf(1025/1024), bf(1)) = (1, 1), both pre1 > 0; so
    # dW2[0] = bf(act1) = (89/64, 1/4), dW1 rows = bf(act0) = (1/2, 0);
    # d act0 = (1, 1) bf(W1) = (97/32, 1), masked by pre0 = (+, -) -> (97/32, 0);
    # dW0[0, 0] = 97/32 bf(515/512) = 97/32 * 129/128, dW0[0, 1] = 97/32 bf(257/256)
    # = 97/32, dW0[0, 26] = 97/32 (1 + 2^-20) (the transceiver feature is exact);
    # d x_mean = 97/32 * (bf(1029/1024), bf(-259/256)) = 97/32 * (129/128, -65/64).
    from fractions import Fraction as F
    from oracle import grad as G
    _, xm, xs, mlp, _ = _mlp_fixture()
    dout = np.zeros((1, 7))
    dout[0, 0] = 1.0
    dW, db, dxm = G.mlp_backward(xm, xs, mlp, dout, bf16=True)
    f = lambda q: float(q)
    np.testing.assert_array_equal(dW[2][0], [89 / 64, 1 / 4])
    np.testing.assert_array_equal(dW[2][1:], 0.0)
    np.testing.assert_array_equal(db[2], dout[0])
    np.testing.assert_array_equal(dW[1], [[0.5, 0.0], [0.5, 0.0]])
    np.testing.assert_array_equal(db[1], [1.0, 1.0])
    expect0 = np.zeros(89)
    expect0[0] = f(F(97, 32) * F(129, 128))
    expect0[1] = f(F(97, 32))
    expect0[26] = f(F(97, 32) * (1 + F(1, 2 ** 20)))
    np.testing.assert_array_equal(dW[0][0], expect0)
    np.testing.assert_array_equal(dW[0][1], 0.0)
    np.testing.assert_array_equal(db[0], [97 / 32, 0.0])
    np.testing.assert_array_equal(dxm[0, :2], [f(F(97, 32) * F(129, 128)), f(F(97, 32) * F(-65, 64))])
    np.testing.assert_array_equal(dxm[0, 2:], 0.0)
