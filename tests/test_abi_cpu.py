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
    assert lib.rsrr_sample_gmres(None, None, 1, None, 1, None, None, None, 1, 1, 1e-10, 8, 10, 0, None, 1, None) == -1
    assert b"gfx950" in lib.rsrr_version()


def test_server_argument_errors_without_device(lib):
    from paper_1605_07951_amd import rsrr
    cfg = rsrr.RsrrServerConfig(0, 1, 0, 0, 0, 0, 1 << 20, 1 << 20, 0, None)  # max_slots = 0
    h = C.c_void_p()
    assert lib.rsrr_server_create(None, C.byref(cfg)) == -1
    assert lib.rsrr_server_create(C.byref(h), None) == -2
    assert lib.rsrr_server_create(C.byref(h), C.byref(cfg)) == -2
    cfg = rsrr.RsrrServerConfig(0, 7, 1, 0, 0, 0, 1 << 20, 1 << 20)  # bad precision
    assert lib.rsrr_server_create(C.byref(h), C.byref(cfg)) == -2
    cfg = rsrr.RsrrServerConfig(0, 1, 1, 0, 0, 0, 0, 1 << 20)  # empty arena
    assert lib.rsrr_server_create(C.byref(h), C.byref(cfg)) == -2
    cfg = rsrr.RsrrServerConfig(0, 1, 1, 0, 9, 0, 1 << 20, 1 << 20)  # too many solve threads
    assert lib.rsrr_server_create(C.byref(h), C.byref(cfg)) == -2
    rid = C.c_int(0)
    assert lib.rsrr_server_submit(None, None, C.byref(rid)) == -1
    assert lib.rsrr_server_wait(None, 1, 0.0, None) == -1
    assert lib.rsrr_server_stats(None, None) == -1
    assert lib.rsrr_server_destroy(None) == -1
    b = C.c_ulonglong(0)
    assert lib.rsrr_server_footprint(None, None, C.byref(b)) == -1
    cfg = rsrr.RsrrServerConfig(0, 1, 1, 0, 0, 0, 1 << 30, 1 << 30)
    assert lib.rsrr_server_footprint(C.byref(cfg), None, C.byref(b)) == -2


def test_server_footprint_is_the_documented_sum(lib):
    """rsrr_server_footprint (host only): S with the reserve columns + kept complex FP32 factors
    (P x P, interchanges, diagonal-block inverses) + Q + V, each rounded up to 256 bytes."""
    from paper_1605_07951_amd import rsrr
    n, N, L, Lx, me = 200, 32, 4, 12, 64
    dummy = (C.c_double * 2)()
    nep = rsrr.RsrrNep(0, n, 3, C.cast(dummy, C.c_void_p), n, C.cast(C.pointer(rsrr.RsrrTerm()), C.POINTER(rsrr.RsrrTerm)),
                       None, 0.0)
    req = rsrr.RsrrRequest(nep, 0.0, 5.0, 4.0, 1.0, N, L, C.cast(dummy, C.c_void_p), n, 0, 0, 0.0, me,
                           C.cast(dummy, C.POINTER(C.c_double)), C.cast(dummy, C.POINTER(C.c_double)), None, Lx, 0)
    al = lambda x: (x + 255) // 256 * 256
    P = 256
    npan = (P + 31) // 32
    for prec, esz, inv in ((1, 8, 2 * 128 * (P + 128) * 8), (0, 16, 0)):
        cfg = rsrr.RsrrServerConfig(0, prec, 1, 0, 0, 0, 1 << 30, 1 << 30)
        b = C.c_ulonglong(0)
        assert lib.rsrr_server_footprint(C.byref(cfg), C.byref(req), C.byref(b)) == 0
        fac = al(N * P * P * esz) + al(N * npan * 2 * 128 * 8) + al(N * inv)
        want = al(n * N * (L + Lx) * 16) + fac + al(n * min(n, N * (L + Lx)) * 16) + al(n * me * 16)
        assert b.value == want


def test_server_structs_match_header(lib):
    """ctypes mirrors of the serving structs have the C sizes (compiled here with gcc)."""
    import subprocess
    import tempfile
    from paper_1605_07951_amd import rsrr
    src = ('#include <stdio.h>\n#include "rsrr.h"\nint main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", '
           'sizeof(rsrr_request), sizeof(rsrr_result), sizeof(rsrr_server_config), sizeof(rsrr_nep), '
           'sizeof(rsrr_instance), sizeof(rsrr_gmres_info), sizeof(rsrr_options), sizeof(rsrr_solve_info), '
           'sizeof(rsrr_point_info)); printf("%zu\\n", sizeof(rsrr_csr)); return 0;}\n')
    with tempfile.TemporaryDirectory() as d:
        cpath, exe = os.path.join(d, "sz.c"), os.path.join(d, "sz")
        open(cpath, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), cpath, "-o", exe], check=True)
        got = [int(x) for x in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    assert got == [C.sizeof(rsrr.RsrrRequest), C.sizeof(rsrr.RsrrResult), C.sizeof(rsrr.RsrrServerConfig),
                   C.sizeof(rsrr.RsrrNep), C.sizeof(rsrr.RsrrInstance), C.sizeof(rsrr.RsrrGmresInfo),
                   C.sizeof(rsrr.RsrrOptions), C.sizeof(rsrr.RsrrSolveInfo), C.sizeof(rsrr.RsrrPointInfo),
                   C.sizeof(rsrr.RsrrCsr)]


def test_options_struct_layout_and_defaults(lib):
    """rsrr_options: every field at the offset the header gives it, size first, and the defaults
    that rsrr_options_init writes; a NULL struct is refused."""
    import subprocess
    import tempfile
    from paper_1605_07951_amd import rsrr
    fields = [f for f, _ in rsrr.RsrrOptions._fields_]
    body = " ".join(f'printf("%zu ", offsetof(rsrr_options, {f}));' for f in fields)
    src = ('#include <stdio.h>\n#include <stddef.h>\n#include "rsrr.h"\n'
           'int main(void){' + body + ' printf("%d\\n", RSRR_OPTIONS_VERSION); return 0;}\n')
    with tempfile.TemporaryDirectory() as d:
        cpath, exe = os.path.join(d, "off.c"), os.path.join(d, "off")
        open(cpath, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), cpath, "-o", exe], check=True)
        got = [int(x) for x in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    assert got[:-1] == [getattr(rsrr.RsrrOptions, f).offset for f in fields]
    assert fields[0] == "size"
    o = rsrr.rsrr_options()
    assert o.size == C.sizeof(rsrr.RsrrOptions) and o.version == got[-1] == 1
    assert (o.ir_max_iters, o.ir_max_iters_batched, o.basis_sketch_max) == (10, 3, 1024)
    assert (o.ir_tol, o.fallback_resid, o.delta, o.tol_gap) == (4.0, 1e-10, 1e-14, 1e3)
    assert lib.rsrr_options_init(None) == -1
    assert lib.rsrr_set_options(None, C.byref(o)) == -1
    assert lib.rsrr_get_options(None, C.byref(o)) == -1
