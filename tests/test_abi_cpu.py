"""CPU checks of the C ABI: the library loads, exports every declared entry
point, computes contour nodes like the oracle, and rejects invalid arguments
before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import rsrr_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsrr.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1605_07951_amd import rsrr
    if not os.path.exists(rsrr.LIB_PATH):
        from paper_1605_07951_amd import build
        build.build()
    return rsrr.lib()


def declared_symbols():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"RSRR_API\s+[\w\s\*]+?\b(rsrr_\w+)\s*\(", txt)))


def test_header_declares_the_four_calls():
    syms = declared_symbols()
    for s in ("rsrr_sample", "rsrr_basis", "rsrr_project", "rsrr_solve"):
        assert s in syms


def test_library_exports_every_declared_symbol(lib):
    for s in declared_symbols():
        assert hasattr(lib, s), s


def test_contour_matches_oracle(lib):
    from paper_1605_07951_amd import rsrr
    for (g, a, b, N) in [(3.8, 1.4, 0.3, 64), (5j, 4.0, 1.0, 32), (-20, 15, 15, 48), (0.0, 1.0, 2.0, 1)]:
        z, w = rsrr.rsrr_contour(g, a, b, N)
        zo, wo = O.ellipse(g, a, b, N)
        assert np.max(np.abs(z - zo)) <= 4e-16 * max(1.0, np.max(np.abs(zo)))
        assert np.max(np.abs(w - wo)) <= 4e-16 * max(1.0, np.max(np.abs(wo)))


def test_argument_errors_without_device(lib):
    dp = C.POINTER(C.c_double)
    z = (C.c_double * 4)()
    assert lib.rsrr_contour(0.0, 0.0, 0.0, 1.0, 2, z, None) == -3
    assert lib.rsrr_contour(0.0, 0.0, 1.0, -1.0, 2, z, None) == -4
    assert lib.rsrr_contour(0.0, 0.0, 1.0, 1.0, 0, z, None) == -5
    assert lib.rsrr_contour(0.0, 0.0, 1.0, 1.0, 2, C.cast(None, dp), None) == -6
    assert lib.rsrr_create(None, 0, None) == -1
    assert lib.rsrr_destroy(None) == -1
    assert lib.rsrr_sample(None, None, 1, None, None, 1, 1, 0, None, 1, None) == -1
    k = C.c_int(0)
    assert lib.rsrr_basis(None, 1, 1, None, 1, 1e-14, None, 1, 1, C.byref(k), None) == -1
    assert lib.rsrr_last_timings(None, None) == -1
    assert lib.rsrr_update_stats(None, 0, 0, None) == -1
    assert b"gfx950" in lib.rsrr_version()
