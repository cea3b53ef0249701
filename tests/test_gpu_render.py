"""GPU parity of the render path (HIP library through the C ABI) against the
FP64 oracle: static render, deformable FP32 render, step oracles (scan, sort,
keys, ranges) and edge cases."""
import numpy as np
import pytest

from oracle import model as M
from paper_2506_12787_amd import synth
from tests import helpers as Hh

pytestmark = pytest.mark.gpu

H0, W0 = 90, 360


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2506_12787_amd import binding
    assert torch.cuda.is_available(), "GPU test on a machine without a GPU"
    c = binding.Context(0)
    yield c
    c.close()


def _tx(b, seed):
    import torch
    return torch.from_numpy(synth.tx_positions(b, seed=seed)).cuda()


def _render_static(ctx, g, H, W, flags=0):
    from paper_2506_12787_amd import binding as B
    sid = ctx.upload_scene(g, H, W)
    out = ctx.render(sid, None, flags=B.NO_DEFORM | flags, batch=1)
    return sid, out[0].cpu().numpy()


def test_static_render_matches_oracle_c0(ctx):
    # N = 2000, 90 x 360, static FP32
    g, s = Hh.problem(2000, H0, W0, seed=1000)
    sid, img = _render_static(ctx, g, H0, W0)
    res, _, _, _ = M.render_query(s, None, None)
    rep = Hh.parity(img, res)
    print("c0 parity", rep)
    assert rep["worst_unflagged_rel"] <= Hh.TOL_REL
    ctx.release_scene(sid)


@pytest.mark.parametrize("H,W,n,seed", [(17, 33, 60, 5), (1, 1, 3, 6), (16, 16, 40, 7), (45, 130, 700, 8)])
def test_static_ragged_grids(ctx, H, W, n, seed):
    g, s = Hh.problem(n, H, W, seed=seed, scale_range=(0.5, 6.0))
    sid, img = _render_static(ctx, g, H, W)
    res, _, _, _ = M.render_query(s, None, None)
    Hh.parity(img, res)
    ctx.release_scene(sid)


def test_empty_and_culled_render_exact_zero(ctx):
    g, _ = Hh.problem(0, 20, 30, seed=1)
    sid, img = _render_static(ctx, g, 20, 30)
    assert np.all(img == 0.0)
    ctx.release_scene(sid)
    g, _ = Hh.problem(50, 20, 30, seed=2)
    g["mean_x"][:] = -200.0
    g["log_scale_y"][:5] = np.nan
    g["depth"][5:10] = np.nan
    sid, img = _render_static(ctx, g, 20, 30)
    assert np.all(img == 0.0)
    ctx.release_scene(sid)


def test_tile8_and_full_sort_are_bitwise_equal(ctx):
    from paper_2506_12787_amd import binding as B
    g, s = Hh.problem(1500, H0, W0, seed=21)
    sid = ctx.upload_scene(g, H0, W0)
    a = ctx.render(sid, None, flags=B.NO_DEFORM, batch=1).cpu().numpy()
    b = ctx.render(sid, None, flags=B.NO_DEFORM | B.TILE8, batch=1).cpu().numpy()
    c = ctx.render(sid, None, flags=B.NO_DEFORM | B.FULL_SORT, batch=1).cpu().numpy()
    d = ctx.render(sid, None, flags=B.NO_DEFORM, batch=1).cpu().numpy()
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(a, c)
    np.testing.assert_array_equal(a, d)  # deterministic
    ctx.release_scene(sid)


def test_speculative_capacity_overflow_renders_again(ctx):
    """A direct render whose key buffer was sized by an earlier, smaller render
    builds its lists at that capacity while the count is read back; when the
    count does not fit it renders again at the exact size. Small scene, then a
    larger one (overflow and re-render), then the small one again (fits): each
    result equals a render of the same scene on a fresh context."""
    from paper_2506_12787_amd import binding as B
    scenes = [Hh.problem(n, H0, W0, seed=90 + n, scale_range=(1.0, 12.0))[0] for n in (300, 6000)]
    got = []
    for g in (scenes[0], scenes[1], scenes[0]):
        sid = ctx.upload_scene(g, H0, W0)
        got.append(ctx.render(sid, None, flags=B.NO_DEFORM, batch=1).cpu().numpy())
        ctx.release_scene(sid)
    fresh = B.Context(0)
    try:
        for g, img in zip((scenes[0], scenes[1], scenes[0]), got):
            sid = fresh.upload_scene(g, H0, W0)
            ref = fresh.render(sid, None, flags=B.NO_DEFORM, batch=1).cpu().numpy()
            np.testing.assert_array_equal(img, ref)
            fresh.release_scene(sid)
    finally:
        fresh.close()
    assert np.abs(got[1]).max() > 0


@pytest.mark.parametrize("n,scale,batch,H,W", [(2500, (1.0, 12.0), 3, 90, 360), (1100, (20.0, 60.0), 2, 90, 360),
                                               (1024, (2.0, 8.0), 1, 90, 360), (1, (1.0, 3.0), 2, 90, 360),
                                               (5000, (1.0, 40.0), 2, 180, 720), (4097, (0.5, 20.0), 3, 250, 1100)])
def test_binned_lists_equal_full_sort(ctx, n, scale, batch, H, W):
    """The binning path (the default) builds the same per-tile lists as the
    full 64-bit (tile, depth) radix sort: counts, keys, values and ranges
    bitwise, and the same images. Large Gaussians put tens of thousands of keys
    into one 256-pair batch (several 2048-key chunks); N is ragged against the
    pair blocks (1024, or 8192 beyond 256 tiles); 180 x 720 (540 tiles, 2
    segments of 512) and 250 x 1100 (1104 tiles, 3 segments) bin segment by
    segment; deformation differs per query."""
    import torch
    from paper_2506_12787_amd import binding as B
    from paper_2506_12787_amd import synth
    T = -(-W // 16) * -(-H // 16)
    g, s = Hh.problem(n, H, W, seed=41 + n, scale_range=scale)
    Ws, bs = synth.mlp_weights(seed=7, out_scale=1.0)
    sid = ctx.upload_scene(g, H, W, mlp=(Ws, bs))
    tx = torch.from_numpy(synth.tx_positions(batch, seed=43)).cuda()
    outs, lists = [], []
    for flags in (B.MLP_FP32, B.MLP_FP32 | B.FULL_SORT):
        outs.append(ctx.render(sid, tx, flags=flags).cpu().numpy())
        lists.append(ctx.debug_keys(batch, n, T))
    a, b = lists
    assert len(a["keys"]) == len(b["keys"]) > 0
    for k in ("counts", "offsets", "keys", "values", "ranges"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    np.testing.assert_array_equal(outs[0], outs[1])
    if scale[0] >= 20.0:
        assert int(a["counts"].max()) > 8  # a 256-pair batch then exceeds one 2048-key chunk
    if T > 256:  # tiles beyond the first segment
        assert int(a["keys"][-1] >> np.uint64(32)) % T >= 256
    ctx.release_scene(sid)


@pytest.mark.parametrize("H,W", [(1024, 1024), (4096, 4096)])
def test_maximum_grids_sampled_pixels(ctx, H, W):
    """The largest grids: 1024 x 1024 is 4096 tiles per query, the most the
    binning path takes (8 segments of 512); 4096 x 4096 (the largest accepted
    size, 65536 tiles) takes the sort path. Static FP32 render, sampled pixels
    against the FP64 oracle; the 1024 grid also against the full sort, bitwise."""
    from paper_2506_12787_amd import binding as B
    g, s = Hh.problem(3000, H, W, seed=61, scale_range=(1.0, 40.0))
    sid = ctx.upload_scene(g, H, W)
    img = ctx.render(sid, None, flags=B.NO_DEFORM, batch=1)[0]
    rng = np.random.default_rng(62)
    px = np.concatenate([rng.integers(0, W, 200), [0, W - 1, 0, W - 1]]).astype(np.int32)
    py = np.concatenate([rng.integers(0, H, 200), [0, 0, H - 1, H - 1]]).astype(np.int32)
    import torch
    gpu = img[torch.from_numpy(py.astype(np.int64)).cuda(), torch.from_numpy(px.astype(np.int64)).cuda()]
    res, _, _, _ = M.render_query(s, None, None, pix=(px, py))
    print(f"{H}x{W}", Hh.parity(gpu.cpu().numpy(), res))
    assert float(img.abs().max()) > 0
    if H * W <= 1024 * 1024:
        full = ctx.render(sid, None, flags=B.NO_DEFORM | B.FULL_SORT, batch=1)[0]
        assert torch.equal(img, full)
    ctx.release_scene(sid)


def _oracle_keys(s, H, W, tile=16):
    gm = M.deform(s, None)
    rg = M.gaussians_for_raster(gm, s.depth)
    rect, flagged, alts = M.tile_rects(gm, rg, H, W, tile)
    return rect, flagged, alts


@pytest.mark.parametrize("full", [False, True])
def test_keys_offsets_ranges_bit_exact(ctx, full):
    from paper_2506_12787_amd import binding as B
    H, W = H0, W0
    g, s = Hh.problem(800, H, W, seed=31)
    sid = ctx.upload_scene(g, H, W)
    ctx.render(sid, None, flags=B.NO_DEFORM | (B.FULL_SORT if full else 0), batch=1)
    TW, TH = -(-W // 16), -(-H // 16)
    dk = ctx.debug_keys(1, s.n, TW * TH)
    rect, flagged, alts = _oracle_keys(s, H, W)
    order = M.depth_order(s.depth)
    assert not flagged.any(), "seeded case chosen without ambiguous rectangles"
    counts = M.rect_count(rect)[order]
    offs, tot = M.exclusive_scan(counts)
    np.testing.assert_array_equal(dk["counts"], counts.astype(np.uint32))
    np.testing.assert_array_equal(dk["offsets"], offs.astype(np.uint32))
    gt, dbits, ids, ranges = M.key_list(rect, s.depth, H, W)
    assert len(dk["keys"]) == tot == len(gt)
    np.testing.assert_array_equal(dk["keys"], (gt << np.uint64(32)) | dbits)
    np.testing.assert_array_equal(dk["values"], ids.astype(np.uint64))
    np.testing.assert_array_equal(dk["ranges"].astype(np.int64), ranges)
    ctx.release_scene(sid)


@pytest.mark.parametrize("n", [0, 1, 255, 256, 257, 4097, 16384, 16385, (1 << 20) + 1])
def test_exclusive_scan_matches_sequential_sum(ctx, n):
    import torch
    rng = np.random.default_rng(n)
    c = rng.integers(0, 200, n).astype(np.uint32)
    off, tot = ctx.exclusive_scan(torch.from_numpy(c.view(np.int32)).cuda())
    ref, rtot = M.exclusive_scan(c)
    assert int(tot.cpu()[0]) == rtot
    np.testing.assert_array_equal(off.cpu().numpy().view(np.uint32), ref.astype(np.uint32))


@pytest.mark.parametrize("n,kind,bits", [
    (0, "rand", 32), (1, "rand", 32), (255, "rand", 32), (256, "rand", 20), (257, "rand", 32),
    (5000, "equal", 32), (5000, "reversed", 16), (100003, "rand", 13), ((1 << 20) + 1, "rand", 32),
    (70000, "rand64", 64), (70000, "rand64", 46)])
def test_radix_sort_matches_stable_sort(ctx, n, kind, bits):
    import torch
    rng = np.random.default_rng(n + bits)
    wide = kind == "rand64"
    dt = np.uint64 if wide else np.uint32
    if kind == "equal":
        k = np.full(n, 7, dt)
    elif kind == "reversed":
        k = np.arange(n, 0, -1).astype(dt) % dt(1 << bits)
    else:
        k = rng.integers(0, 1 << min(bits, 63), n, dtype=np.uint64).astype(dt)
        if wide and bits == 64:
            k = k ^ (rng.integers(0, 2, n, dtype=np.uint64) << np.uint64(63))
    v = np.arange(n, dtype=np.uint32)
    tk = torch.from_numpy(k.view(np.int64 if wide else np.int32).copy()).cuda()
    tv = torch.from_numpy(v.view(np.int32).copy()).cuda()
    ctx.radix_sort(tk, tv, 0, bits)
    o = np.argsort(k & dt((1 << bits) - 1) if bits < 64 else k, kind="stable")
    np.testing.assert_array_equal(tk.cpu().numpy().view(dt), k[o])
    np.testing.assert_array_equal(tv.cpu().numpy().view(np.uint32), v[o])


def _deform_problem(n, B, seed, out_scale, n_hidden=4):
    g, s = Hh.problem(n, H0, W0, seed=seed)
    Ws, bs = synth.mlp_weights(seed=seed + 2000, out_scale=out_scale, n_hidden=n_hidden)
    rng = np.random.default_rng(seed)
    bs = [b + rng.normal(0, 0.05, b.shape).astype(np.float32) for b in bs]
    return g, s, Ws, bs


@pytest.mark.parametrize("n_hidden", [4, 3, 2, 1])
def test_deform_residuals_fp32_match_oracle(ctx, n_hidden):
    # depths 1..4: no hidden-to-hidden layer, one (the odd tail of the kernel's two-layer loop), two (the loop
    # only) and three (loop and tail); 4 x 3001 pairs leave a ragged last wave (4 of its 16 pairs)
    g, s, Ws, bs = _deform_problem(3001, 4, seed=41 + n_hidden, out_scale=1.0, n_hidden=n_hidden)
    sid = ctx.upload_scene(g, H0, W0, mlp=(Ws, bs))
    tx = _tx(4, 2041)
    d = ctx.debug_deform(sid, tx).cpu().numpy().astype(np.float64)
    mlp = Hh.mlp_f64(Ws, bs)
    txh = tx.cpu().numpy().astype(np.float64)
    worst = 0.0
    for b in range(4):
        ref = M.deltas(s, mlp, txh[b])
        scale = np.abs(ref).max(axis=0)
        err = np.abs(d[b] - ref).max(axis=0) / scale
        worst = max(worst, err.max())
    print(f"FP32 MLP residual normwise rel err (depth {n_hidden})", worst)
    assert worst < 2e-5
    ctx.release_scene(sid)


@pytest.mark.parametrize("out_scale", [0.01, 1.0])
def test_deformable_fp32_render_matches_oracle(ctx, out_scale):
    g, s, Ws, bs = _deform_problem(2000, 3, seed=51, out_scale=out_scale)
    sid = ctx.upload_scene(g, H0, W0, mlp=(Ws, bs))
    tx = _tx(3, 2051)
    out = ctx.render(sid, tx).cpu().numpy()
    mlp = Hh.mlp_f64(Ws, bs)
    txh = tx.cpu().numpy().astype(np.float64)
    for b in range(3):
        res, _, _, _ = M.render_query(s, mlp, txh[b])
        rep = Hh.parity(out[b], res)
        print("deform parity", out_scale, b, rep)
    ctx.release_scene(sid)
