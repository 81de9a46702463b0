"""Pins of the incremental-round oracle and of the round schedule (CPU only).

Expected distance: closed forms (isotropic: sigma sqrt(pi/2); one axis: the
half-normal mean) and Monte Carlo; the library's own quadrature agrees.  Tile
sets: the containment that Eq. 3 / Eq. 4 guarantee, the coverage of Eq. 5,
disjoint rounds whose union holds the final fovea, and key counts of a tile
set against a per-Gaussian brute force.
"""
import math

import numpy as np
import pytest

import oracle.core as oc
import oracle.incremental as oi
import synth


def test_expected_distance_closed_forms():
    for s in (0.5, 3.0, 117.0):
        assert oi.expected_distance(s, s) == pytest.approx(s * math.sqrt(math.pi / 2.0), rel=1e-14)
        assert oi.expected_distance(s, 0.0) == pytest.approx(s * math.sqrt(2.0 / math.pi), rel=1e-14)
    assert oi.expected_distance(0.0, 0.0) == 0.0


def test_expected_distance_monte_carlo():
    rng = np.random.default_rng(3)
    for sx, sy in ((234.3, 260.7), (10.0, 1.0), (2.0, 5.0)):
        z = rng.normal(size=(2, 2_000_000))
        d = np.hypot(sx * z[0], sy * z[1])
        se = d.std() / math.sqrt(d.size)
        assert abs(oi.expected_distance(sx, sy) - d.mean()) < 4 * se


def test_schedule_quadrature_matches_oracle():
    from paper_2507_04147_amd import incremental as inc
    for sx, sy in ((234.3, 260.7), (99.3, 93.7), (1.0, 40.0), (5.0, 5.0)):
        assert inc.expected_distance(sx, sy) == pytest.approx(oi.expected_distance(sx, sy), rel=1e-12)
    assert inc.round_radius(274.8, 300.0) == 0.0
    assert inc.round_radius(274.8, 100.0) == pytest.approx(174.8)
    assert inc.speculative_radius(274.8, 100.0) == pytest.approx(374.8)


def _cam():
    return synth.foveated_stereo(n=10)[1][0]


def test_eq3_containment_on_tiles():
    """r_i = max(0, r_N - dist(u_i, u_N)) keeps C_i's tiles inside C_N's."""
    cam = _cam()
    rng = np.random.default_rng(5)
    for _ in range(60):
        uN = rng.uniform((0, 0), (cam.width, cam.height))
        ui = uN + rng.normal(0.0, 150.0, 2)
        rN = rng.uniform(50.0, 400.0)
        ri = max(0.0, rN - float(np.hypot(*(ui - uN))))
        a, b = oi.disc_tiles(cam, ui, ri), oi.disc_tiles(cam, uN, rN)
        assert not np.any(a & (1 - b))


def test_eq5_coverage_on_tiles():
    """r_max = r_f + E covers C_N whenever dist(u_j, u_N) <= E."""
    cam = _cam()
    rng = np.random.default_rng(6)
    rf = 274.8
    for _ in range(60):
        uN = rng.uniform((0, 0), (cam.width, cam.height))
        E = rng.uniform(20.0, 300.0)
        ang, dist = rng.uniform(0, 2 * math.pi), rng.uniform(0.0, E)
        uj = uN + dist * np.array([math.cos(ang), math.sin(ang)])
        a, b = oi.disc_tiles(cam, uj, oi.speculative_radius(rf, E)), oi.disc_tiles(cam, uN, rf)
        assert not np.any(b & (1 - a))


def test_round_tiles_partition_and_cover():
    cam = _cam()
    trials, sig = synth.gaze_exits(n_trials=3)
    rf = 0.15 * cam.width
    for final, exits in trials:
        rounds = []
        for gz, (sx, sy) in zip(exits, sig):
            e = oi.expected_distance(sx, sy)
            rounds += [(gz[0], oi.round_radius(rf, e)), (gz[0], oi.speculative_radius(rf, e))]
        news, union = oi.round_tiles(cam, rounds, final[0], rf)
        tot = np.zeros_like(union)
        for nw in news:
            assert not np.any(tot & nw)  # disjoint
            tot |= nw
        assert np.array_equal(tot, union)
        need = oi.disc_tiles(cam, final[0], rf)
        assert not np.any(need & (1 - union))  # the final fovea is covered after the last round
        # the last round renders exactly what the earlier rounds left of C_N
        before = tot & (1 - news[-1])
        assert np.array_equal(news[-1], need & (1 - before))


def test_keys_for_tiles_brute_force():
    sc = synth.make_scene(400, 1.0, seed=8)
    cam = synth.make_camera(96, 80, 60.0, (0.0, 0.0, -3.0))
    v = oc.full_view(cam)
    pr = oc.project(sc, [v])
    tx, ty = (96 + 15) // 16, (80 + 15) // 16
    rng = np.random.default_rng(9)
    tiles = (rng.uniform(size=tx * ty) < 0.4).astype(np.uint8)
    want = 0
    for i in np.nonzero(pr["vis"][0])[0]:
        x0, x1, y0, y1 = pr["rect"][0, i]
        for yy in range(y0, y1 + 1):
            for xx in range(x0, x1 + 1):
                want += int(tiles[yy * tx + xx])
    assert oi.keys_for_tiles(pr["rect"][0], pr["vis"][0], tiles, tx, ty) == want
    # every tile: the plain render's key count
    assert oi.keys_for_tiles(pr["rect"][0], pr["vis"][0], np.ones(tx * ty, np.uint8), tx, ty) == \
        int(pr["count"][0][pr["vis"][0].astype(bool)].sum())
