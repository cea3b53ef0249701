"""Serving loop (continuous batching, captured graphs, admission by memory):
each result is bitwise identical alone and in a mixed stream, per-scene
batches and batches across scenes (mixed mode, graphs keyed by capacities),
under forced shrinking and forced key overflow; error paths."""
import numpy as np
import pytest

from paper_2506_12787_amd import synth
from tests import helpers as Hh

pytestmark = pytest.mark.gpu

SCENES = [(3000, 90, 360), (2000, 180, 720), (6000, 90, 360)]


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_2506_12787_amd import binding as B
    assert torch.cuda.is_available()
    c = B.Context(0)
    sids = []
    for i, (n, H, W) in enumerate(SCENES):
        g = synth.gaussians(n, H, W, seed=500 + i)
        Ws, bs = synth.mlp_weights(seed=600 + i, out_scale=1.0)
        sids.append(c.upload_scene(g, H, W, mlp=(Ws, bs)))
    rng = np.random.default_rng(9)
    reqs = [(int(rng.integers(0, len(SCENES))), synth.tx_positions(1, seed=700 + k)[0]) for k in range(48)]
    alone = []
    for si, tx in reqs:
        t = torch.from_numpy(tx[None].copy()).cuda()
        alone.append(c.render(sids[si], t, flags=B.MLP_BF16)[0].cpu().numpy())
    yield c, sids, reqs, alone
    c.close()


def _serve_all(c, sids, reqs, **cfg):
    c.serve_start(**cfg)
    outs, tks = [], []
    for si, tx in reqs:
        n, H, W = SCENES[si]
        o = np.zeros((H, W), np.float32)
        tks.append(c.serve_submit(sids[si], tx, o))
        outs.append(o)
    stats = [c.serve_wait(t) for t in tks]
    cnt = c.serve_counters()
    c.serve_stop()
    return outs, stats, cnt


@pytest.mark.parametrize("graphs", [True, False])
def test_mixed_stream_equals_alone(setup, graphs):
    c, sids, reqs, alone = setup
    outs, stats, cnt = _serve_all(c, sids, reqs, max_batch=8, n_slots=2, use_graphs=graphs, mixed=False)
    for o, a in zip(outs, alone):
        np.testing.assert_array_equal(o, a)
    assert cnt["completed"] == len(reqs)
    assert max(s["batch"] for s in stats) > 1  # requests were actually batched
    if graphs:
        assert cnt["graph_builds"] >= 1
    print("counters", cnt)


@pytest.mark.parametrize("graphs", [True, False])
def test_mixed_mode_batches_across_scenes(setup, graphs):
    # one launch holds requests of several scenes (different sizes, grids and MLPs); every result is what the
    # query renders alone, and a handful of capacity-keyed graphs serves all the batches
    c, sids, reqs, alone = setup
    outs, stats, cnt = _serve_all(c, sids, reqs, max_batch=16, n_slots=2, use_graphs=graphs, mixed=True)
    for i, (o, a) in enumerate(zip(outs, alone)):
        np.testing.assert_array_equal(o, a, err_msg=f"request {i}")
    assert cnt["completed"] == len(reqs)
    assert cnt["mixed_launches"] == cnt["launches"] >= 1
    assert cnt["mixed_scenes"] > cnt["mixed_launches"]  # some launch held more than one scene
    assert max(s["batch"] for s in stats) > 1
    if graphs:
        assert 1 <= cnt["graph_builds"] <= 2 * cnt["launches"]
    print("counters", cnt)


def test_mixed_mode_fp32_batches_across_scenes(setup):
    # a server at the paper's precision (FP32 MLP) batches across scenes too; every result is what the query renders
    # alone with the FP32 MLP
    import torch
    from paper_2506_12787_amd import binding as B
    c, sids, reqs, _ = setup
    alone32 = []
    for si, tx in reqs:
        t = torch.from_numpy(tx[None].copy()).cuda()
        alone32.append(c.render(sids[si], t, flags=B.MLP_FP32)[0].cpu().numpy())
    outs, stats, cnt = _serve_all(c, sids, reqs, max_batch=16, n_slots=2, flags=B.MLP_FP32, mixed=True)
    for i, (o, a) in enumerate(zip(outs, alone32)):
        np.testing.assert_array_equal(o, a, err_msg=f"request {i}")
    assert cnt["completed"] == len(reqs)
    assert cnt["mixed_launches"] == cnt["launches"] >= 1
    assert cnt["mixed_scenes"] > cnt["mixed_launches"]
    print("counters", cnt)


def test_mixed_mode_keeps_static_scenes_apart(setup):
    # a scene without an MLP renders statically: it never shares a launch with the deformable scenes, and its
    # requests still come back right
    import torch
    from paper_2506_12787_amd import binding as B
    c, sids, reqs, alone = setup
    g = synth.gaussians(1500, 45, 130, seed=510)
    sid_s = c.upload_scene(g, 45, 130)
    ref = c.render(sid_s, None, flags=B.NO_DEFORM, batch=1)[0].cpu().numpy()
    c.serve_start(max_batch=16, n_slots=2, mixed=True)
    outs, tks = [], []
    for k, (si, tx) in enumerate(reqs[:20]):
        for sid, shape in ((sids[si], SCENES[si][1:]), (sid_s, (45, 130))):
            if sid == sid_s and k % 3:
                continue
            o = np.zeros(shape, np.float32)
            tks.append((c.serve_submit(sid, tx, o), sid, k))
            outs.append(o)
    stats = [c.serve_wait(t) for t, _, _ in tks]
    cnt = c.serve_counters()
    c.serve_stop()
    for o, (_, sid, k) in zip(outs, tks):
        np.testing.assert_array_equal(o, ref if sid == sid_s else alone[k])
    assert cnt["completed"] == len(tks) and cnt["mixed_launches"] == cnt["launches"]
    c.release_scene(sid_s)
    torch.cuda.synchronize()
    print("counters", cnt, "batches", sorted({s["batch"] for s in stats}))


def test_mixed_mode_under_budget_and_key_overflow(setup):
    c, sids, reqs, alone = setup
    # one slot: half of what it holds unconstrained forces the 16-query batches to shrink
    _, _, cnt = _serve_all(c, sids, reqs, max_batch=16, n_slots=1, mixed=True)
    budget = cnt["workspace_bytes"] // 2
    outs, stats, cnt = _serve_all(c, sids, reqs, max_batch=16, n_slots=1, hbm_budget=budget, mixed=True)
    for o, a in zip(outs, alone):
        np.testing.assert_array_equal(o, a)
    assert cnt["budget_shrinks"] >= 1 and cnt["workspace_bytes"] <= budget, (cnt, budget)
    outs, stats, cnt = _serve_all(c, sids, reqs[:12], max_batch=4, n_slots=2, key_factor=0.05, mixed=True)
    for o, a in zip(outs, alone[:12]):
        np.testing.assert_array_equal(o, a)
    assert cnt["fallbacks"] >= 1 and any(s["fallback"] for s in stats)
    print("counters", cnt)


def test_memory_budget_shrinks_batches(setup):
    c, sids, reqs, alone = setup
    # a 16-query batch of the largest scene needs ~30 MB: 24 MB forces shrinking
    budget = 24 << 20
    outs, stats, cnt = _serve_all(c, sids, reqs, max_batch=16, n_slots=2, hbm_budget=budget, mixed=False)
    for o, a in zip(outs, alone):
        np.testing.assert_array_equal(o, a)
    assert cnt["budget_shrinks"] >= 1
    assert cnt["workspace_bytes"] <= budget
    print("counters", cnt)


def test_key_overflow_falls_back_to_exact_sizing(setup):
    c, sids, reqs, alone = setup
    outs, stats, cnt = _serve_all(c, sids, reqs[:12], max_batch=4, n_slots=2, key_factor=0.05, mixed=False)
    for o, a in zip(outs, alone[:12]):
        np.testing.assert_array_equal(o, a)
    assert cnt["fallbacks"] >= 1 and any(s["fallback"] for s in stats)


def test_request_errors(setup):
    from paper_2506_12787_amd import binding as B
    c, sids, reqs, alone = setup
    c.serve_start(max_batch=4)
    o = np.zeros((90, 360), np.float32)
    with pytest.raises(B.SwfError):
        c.serve_submit(12345, [1, 1, 1], o)
    with pytest.raises(B.SwfError):
        c.serve_submit(sids[0], [np.nan, 1, 1], o)
    c.serve_stop()
    # a budget below one query of the scene: the request fails, nothing hangs
    c.serve_start(max_batch=4, hbm_budget=1 << 20)
    tk = c.serve_submit(sids[2], [1, 2, 1], o)
    with pytest.raises(B.SwfError):
        c.serve_wait(tk)
    c.serve_stop()
