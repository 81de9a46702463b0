"""FP64 CPU oracle for the foveated 3DGS rendering path (TEST INFRASTRUCTURE).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It shares no code with the HIP library: the C file next to this one is
compiled with gcc (no FP contraction) and called through ctypes, and the
composition of foveated views is written here in Python floats (IEEE doubles).

Parity pins: see tests/test_oracle_*.py; every oracle function is pinned there
against a closed form, an invariant, brute force or an independent library
routine (scipy's spherical harmonics, torch's bilinear interpolation, numpy's
argsort, finite differences).
"""
from .core import *  # noqa: F401,F403
