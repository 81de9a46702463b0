"""The early-exit gaze network stand-in (CPU): one prediction per block, pruning
shrinks the token set by the stated fraction, seeded weights are
deterministic, and the exits come out in order."""
import pytest

torch = pytest.importorskip("torch")

from paper_2507_04147_amd import gaze_vit as gv  # noqa: E402


def _img():
    return torch.rand(1, 1, 96, 160, generator=torch.Generator().manual_seed(1))


def test_exits_and_shapes():
    m = gv.EarlyExitViT(img=(96, 160), dim=48, heads=6)
    outs = list(m.exits_iter(_img()))
    assert [l for l, _ in outs] == [1, 2, 3, 4, 5, 6]
    assert all(g.shape == (1, 2) for _, g in outs)


def test_seeded_and_pruning_changes_only_later_exits():
    a = [g for _, g in gv.EarlyExitViT(img=(96, 160), dim=48, heads=6, seed=3).exits_iter(_img())]
    b = [g for _, g in gv.EarlyExitViT(img=(96, 160), dim=48, heads=6, seed=3).exits_iter(_img())]
    p = [g for _, g in gv.EarlyExitViT(img=(96, 160), dim=48, heads=6, seed=3, prune=0.2).exits_iter(_img())]
    assert all(torch.equal(x, y) for x, y in zip(a, b))
    assert torch.equal(a[0], p[0])          # pruning acts after a block: the first exit is unchanged
    assert not torch.equal(a[-1], p[-1])


def test_pruned_token_counts():
    m = gv.EarlyExitViT(img=(96, 160), dim=48, heads=6, prune=0.1)
    seen = []
    for blk in m.blocks:
        blk.register_forward_hook(lambda mod, inp, out: seen.append(inp[0].shape[1]))
    list(m.exits_iter(_img()))
    n = 6 * 10  # 96/16 x 160/16 patches
    want = [n + 1]
    for _ in range(5):
        want.append(max(1, round((want[-1] - 1) * 0.9)) + 1)
    assert seen == want


def test_exit_latencies_increase():
    lat = gv.exit_latencies(gv.EarlyExitViT(img=(96, 160), dim=48, heads=6), _img(), reps=3)
    assert len(lat) == 6 and all(b >= a for a, b in zip(lat, lat[1:]))
