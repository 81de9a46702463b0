"""Blend variants and the autotuner (MI355X only): every variant (LDS batch
depth, lane pixel block, grid or longest-first queue schedule) gives the same
image, T and last-contributor index bit for bit, on a ragged foveated stereo
frame and on the full-size frame; the autotuner's choice is one of them."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import paper_2507_04147_amd as p
    p.lib()
    assert torch.cuda.is_available()
    return p


def _check_all_variants(pkg, n, W, H, seed):
    scene, cams = synth.foveated_stereo(n=n, width=W, height=H, seed=seed)
    gz = [(c.cx + 13.0, c.cy - 7.0) for c in cams]
    fov = pkg.fovea_struct(0.15 * W, 0.35 * W)
    ctx = pkg.Context()
    ds = pkg.DeviceScene.from_host(scene)
    views = pkg.make_foveated_views(cams, gz, fov)
    ctx.preprocess(ds, views, (3, 10))
    ctx.bin_sort()
    npx = sum(v.width * v.height for v in views)
    ref = None
    for k in range(pkg.BLEND_VARIANTS):
        rgb = torch.full((3 * npx,), float("nan"), device="cuda")
        T = torch.full((npx,), float("nan"), device="cuda")
        last = torch.zeros(npx, dtype=torch.int32, device="cuda")
        ctx.set_blend_variant(k)
        ctx.blend(rgb, T, last)
        ctx.sync()
        act = ctx.inspect("active", torch.uint8)
        out = (rgb.cpu().numpy(), T.cpu().numpy(), last.cpu().numpy())
        if ref is None:
            ref = out
            # every pixel of an active tile was written
            assert np.isfinite(out[1]).sum() > 0
        else:
            for a, b in zip(out, ref):
                np.testing.assert_array_equal(a, b, err_msg=str(pkg.blend_variant_desc(k)))
    ms, best = ctx.autotune_blend(reps=2)
    print("variant ms:", {pkg.blend_variant_desc(k): round(m, 4) for k, m in enumerate(ms)}, "best",
          pkg.blend_variant_desc(best), flush=True)
    assert 0 <= best < pkg.BLEND_VARIANTS and min(ms) == ms[best]
    rgb = torch.full((3 * npx,), float("nan"), device="cuda")
    ctx.blend(rgb)
    ctx.sync()
    np.testing.assert_array_equal(rgb.cpu().numpy(), ref[0])
    ctx.close()


def test_variants_identical_ragged(pkg):
    _check_all_variants(pkg, 60_000, 236, 244, 9)


def test_variants_identical_full_size(pkg):
    _check_all_variants(pkg, 1_000_000, 1832, 1920, 2)
