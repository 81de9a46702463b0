"""The allocation-free entry point (a3fr_region_sse_noalloc) against the
entry point it is a variant of (a3fr_region_sse), through the C ABI: the
same sums and counts bit for bit, on two calls in a row (the second with a
smaller image, so the shared scratch holds the first call's partials when it
starts), and oversize or bad arguments rejected with nothing enqueued."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import paper_2507_04147_amd as p
    p.lib()
    assert torch.cuda.is_available()
    return p


def _images(rng, W, H):
    a = rng.uniform(-0.2, 1.2, (3, H, W)).astype(np.float32)
    b = np.clip(a + rng.normal(0.0, 0.05, a.shape), -0.1, 1.1).astype(np.float32)
    return torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()


def test_noalloc_region_sse_equals_region_sse(pkg):
    rng = np.random.default_rng(7)
    ctx = pkg.Context()
    for W, H, gaze in ((1832, 1920, (916.0, 960.0)), (232, 120, (40.5, 100.25))):
        a, b = _images(rng, W, H)
        rad = (0.15 * W, 0.35 * W)
        want_sse, want_cnt = ctx.region_sse(W, H, gaze, rad[0], rad[1], a, b)
        sse = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
        cnt = torch.full((3,), -1, dtype=torch.int64, device="cuda")
        ctx.region_sse_noalloc(W, H, gaze, rad[0], rad[1], a, b, sse, cnt)
        ctx.sync()
        np.testing.assert_array_equal(cnt.cpu().numpy(), want_cnt)
        np.testing.assert_array_equal(sse.cpu().numpy().view(np.uint64), want_sse.view(np.uint64))
        assert int(want_cnt.sum()) == W * H
    ctx.close()


def test_noalloc_region_sse_rejects_bad_sizes(pkg):
    ctx = pkg.Context()
    a = torch.zeros(3 * 4 * 4, device="cuda")
    sse = torch.zeros(3, dtype=torch.float64, device="cuda")
    cnt = torch.zeros(3, dtype=torch.int64, device="cuda")
    for W, H in ((0, 4), (4, -1), (65536, 65536)):
        with pytest.raises(pkg.A3FRError) as e:
            ctx.region_sse_noalloc(W, H, (0.0, 0.0), 1.0, 2.0, a, a, sse, cnt)
        assert e.value.status == pkg.A3FR_EINVAL
    ctx.sync()
    ctx.close()
