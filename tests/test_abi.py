"""The C-ABI library builds for gfx950, loads on the CPU and exports every
entry point that include/a3fr.h declares (no compute calls: CPU only)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "a3fr.h")).read()
    return sorted(set(re.findall(r"^\s*(?:a3fr_status|void|const char \*)\s*(a3fr_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for must in ("a3fr_preprocess", "a3fr_bin_sort", "a3fr_blend", "a3fr_render_foveated", "a3fr_render_full"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2507_04147_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        from paper_2507_04147_amd import build
        build.build(verbose=False)
    L = pkg.lib()
    missing = [n for n in declared_symbols() if not hasattr(L, n)]
    assert not missing, missing
    assert set(pkg.EXPORTED) <= set(declared_symbols())


def test_status_strings_and_null_context():
    import ctypes as C
    import paper_2507_04147_amd as pkg
    L = pkg.lib()
    assert L.a3fr_status_str(0) == b"ok"
    assert L.a3fr_status_str(1) == b"invalid argument"
    # a NULL context is rejected without touching the device
    assert L.a3fr_preprocess(None, None, None, 0, 0, 0) == pkg.A3FR_EINVAL
    assert L.a3fr_bin_sort(None, None) == pkg.A3FR_EINVAL
    assert L.a3fr_blend(None, None, None, None) == pkg.A3FR_EINVAL


def test_make_foveated_views_matches_oracle_views():
    """The library's layer views (host helper) equal the oracle's, field by field
    (bit-for-bit doubles: the mask radii decide tile sets)."""
    import numpy as np
    import oracle
    import synth
    import paper_2507_04147_amd as pkg
    cams = synth.stereo_cameras((0, 0, -3), 1832, 1920, 60)
    gz = [(900.25, 1000.5), (1100.0, 700.125)]
    rad = (0.15 * 1832, 0.35 * 1832)
    ours = pkg.make_foveated_views(cams, gz, pkg.fovea_struct(*rad))
    ref = oracle.foveated_views(cams, gz, rad)
    assert len(ours) == len(ref) == 6
    for a, b in zip(ours, ref):
        for f in ("fx", "fy", "cx", "cy", "width", "height", "eye", "mask", "select", "gx", "gy", "r_in", "r_out"):
            assert getattr(a, f) == getattr(b, f), f
        assert list(a.R) == list(np.asarray(b.R).reshape(9)) and list(a.t) == list(b.t)
