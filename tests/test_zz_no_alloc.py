"""The allocation-free scan entry point (swf_exclusive_scan_noalloc, static
device scratch) against the allocating one (swf_exclusive_scan), bit-exact,
through the C ABI: two calls in a row, the second with a smaller input, so
that block sums left in the shared scratch by the first call cannot leak into
the second; also the largest scan grid (4096 blocks) and the empty input."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture()
def ctx():
    import torch
    from paper_2506_12787_amd import binding
    assert torch.cuda.is_available(), "GPU test on a machine without a GPU"
    c = binding.Context(0)
    yield c
    c.close()


def _scan_both(ctx, c):
    import torch
    counts = torch.from_numpy(c.view(np.int32)).cuda()
    ref_off, ref_tot = ctx.exclusive_scan(counts)
    off = torch.full((max(len(c), 1),), -1, dtype=torch.int32, device="cuda")
    tot = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    ctx.exclusive_scan_noalloc(counts, off, tot)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(off[:len(c)].cpu().numpy(), ref_off.cpu().numpy())
    assert int(tot.cpu()[0]) == int(ref_tot.cpu()[0])
    return int(tot.cpu()[0])


@pytest.mark.parametrize("sizes", [(9_000_003, 1000), (300_001, 5), (4097, 0)])
def test_noalloc_scan_equals_allocating_scan(ctx, sizes):
    rng = np.random.default_rng(sizes[0])
    for n in sizes:
        c = rng.integers(0, 200, n).astype(np.uint32)
        print(f"noalloc scan n={n}", flush=True)
        tot = _scan_both(ctx, c)
        assert tot == int(c.astype(np.uint64).sum())
