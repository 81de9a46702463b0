"""GPU parity of the AMR levels (MI355X only).

Rendered positions are the plain full-resolution render's pixels and the
other positions copies of them, so the AMR image must equal the GPU's own
full-resolution render gathered by the oracle's level and inheritance rule
bit for bit, and the oracle's AMR image within the colour tolerances
(ambiguous pixels of the plain render, gathered the same way, within 1e-4 plus
the tolerance the oracle derives for each)."""
import numpy as np
import pytest

import oracle.amr as oa
import synth
from test_gpu_parity import COLOUR_TOL, assert_amb_within

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import paper_2507_04147_amd as p
    p.lib()
    assert torch.cuda.is_available()
    return p


def _gpu(pkg, scene, cams, gz, radii):
    ds = pkg.DeviceScene.from_host(scene)
    ctx = pkg.Context()
    H, W = cams[0].height, cams[0].width
    out = torch.full((len(cams), 3, H, W), float("nan"), device="cuda")
    ctx.render_amr(ds, cams, gz, pkg.amr_struct(*radii), out)
    full = torch.empty_like(out)
    ctx.render_full(ds, cams, full)
    ctx.sync()
    ctx.close()
    return out.cpu().numpy(), full.cpu().numpy()


@pytest.mark.parametrize("radii", [(60.0, 110.0, 170.0), (0.0, 0.0, 0.0), (1e9, 1e9, 1e9)])
def test_amr_small_vs_full_render_and_oracle(pkg, radii):
    W, H = 236, 244
    scene, cams = synth.foveated_stereo(n=60_000, width=W, height=H, seed=9)
    gz = [(0.4 * W, 0.55 * H), (0.4 * W + 3.0, 0.55 * H)]
    amr, full = _gpu(pkg, scene, cams, gz, radii)
    for e in range(2):
        lv = oa.tile_levels(cams[e], gz[e], radii)
        assert np.array_equal(amr[e], oa.amr_image(full[e], lv, W, H))
    ref = oa.render_amr(scene, cams, gz, radii)
    for e in range(2):
        lv = oa.tile_levels(cams[e], gz[e], radii)
        amb = oa.amr_image(ref["images"][e]["amb"][None].astype(np.float64), lv, W, H)[0] != 0
        tol = oa.amr_image(ref["images"][e]["amb_tol"][None], lv, W, H)[0]
        err = np.abs(amr[e] - ref["amr"][e])
        assert err.max(axis=0)[~amb].max() <= COLOUR_TOL
        assert_amb_within(err, amb, tol)


def test_amr_full_size(pkg):
    """1M Gaussians, 2 x 1832 x 1920, levels at the fovea, between, mid and beyond."""
    scene, cams = synth.foveated_stereo()
    W, H = cams[0].width, cams[0].height
    gz = [(c.cx, c.cy) for c in cams]
    radii = (0.15 * W, 0.25 * W, 0.35 * W)
    amr, full = _gpu(pkg, scene, cams, gz, radii)
    for e in range(2):
        assert np.array_equal(amr[e], oa.amr_image(full[e], oa.tile_levels(cams[e], gz[e], radii), W, H))


def test_amr_arguments(pkg):
    scene, cams = synth.foveated_stereo(n=1000, width=64, height=64, seed=9)
    ds = pkg.DeviceScene.from_host(scene)
    ctx = pkg.Context()
    out = torch.empty((2, 3, 64, 64), device="cuda")
    gz = [(32.0, 32.0)] * 2
    for bad in ((10.0, 5.0, 20.0), (-1.0, 5.0, 20.0), (1.0, 2.0, float("inf"))):
        with pytest.raises(pkg.A3FRError) as e:
            ctx.render_amr(ds, cams, gz, pkg.amr_struct(*bad), out)
        assert e.value.status == pkg.A3FR_EINVAL
    ctx.close()
