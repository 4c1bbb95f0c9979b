"""The C ABI library loads and exports what include/cfie.h declares (CPU only)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cfie.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cfie_[A-Za-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    from paper_2203_13283_amd import _lib
    assert _declared() == sorted(_lib.EXPORTED)


def test_library_exports_every_declared_symbol():
    import paper_2203_13283_amd as P
    lib = P.load_library()
    for name in _declared():
        assert hasattr(lib, name), name


def test_default_options_and_status_strings():
    from paper_2203_13283_amd import _lib
    o = _lib.default_options()
    assert (o.precision, o.block, o.quad_far, o.quad_near, o.near_band) == (0, 128, 5, 10, 6)
    assert o.compress_tol == 1e-10 and o.fail_alloc_after == -1
    lib = _lib.load()
    assert lib.cfie_status_string(0) == b"ok"
    assert lib.cfie_status_string(100).startswith(b"warning")


def test_create_rejects_bad_options_before_touching_a_device():
    import ctypes
    from paper_2203_13283_amd import _lib
    lib = _lib.load()
    o = _lib.default_options()
    o.block = 0
    h = ctypes.c_void_p()
    assert lib.cfie_create(ctypes.byref(o), 0, None, ctypes.byref(h)) == _lib.CFIE_EINVAL
    assert b"block" in lib.cfie_last_error(None)
    o = _lib.default_options()
    o.quad_far = 7
    assert lib.cfie_create(ctypes.byref(o), 0, None, ctypes.byref(h)) == _lib.CFIE_EINVAL
    o = _lib.default_options()
    assert o.test_matrix == _lib.SKETCH_SRFT
    o.test_matrix = 2
    assert lib.cfie_create(ctypes.byref(o), 0, None, ctypes.byref(h)) == _lib.CFIE_EINVAL
    assert b"test_matrix" in lib.cfie_last_error(None)
    assert lib.cfie_create(None, 0, None, None) == _lib.CFIE_EINVAL
    # NULL context handling of every entry point
    assert lib.cfie_factor(None) == _lib.CFIE_EINVAL
    assert lib.cfie_solve(None, None, 0, None, 0, 0) == _lib.CFIE_EINVAL
    assert lib.cfie_srft_rows(None, None, 0, 0, None, None, 0) == _lib.CFIE_EINVAL
    lib.cfie_destroy(None)


def test_srft_frequency_map():
    """Position -> frequency of the row transform's radix passes (host function).  One pass
    (N <= 32) leaves the natural order; two passes of 2^b1 and 2^b2 points leave frequency
    j = e1 + 2^b1 e2 at position p = 2^b2 e1 + e2 (the digits swapped); in general the map is
    a permutation of [0, N) that is its own inverse when all passes have the same radix."""
    from paper_2203_13283_amd import _lib
    lib = _lib.load()
    f = lib.cfie_srft_frequency
    for n in (8, 16, 32):
        assert [f(n, p) for p in range(n)] == list(range(n))
    # N = 64: passes of 8 and 8; N = 128: passes of 8 and 16
    for n, b1, b2 in ((64, 3, 3), (128, 3, 4), (1024, 5, 5)):
        for p in range(n):
            e1, e2 = p >> b2, p & ((1 << b2) - 1)
            assert f(n, p) == e1 + (e2 << b1), (n, p)
    for n in (2048, 16384, 32768):
        js = [f(n, p) for p in range(n)]
        assert sorted(js) == list(range(n))
    assert [f(16384, f(16384, p)) for p in range(0, 16384, 37)] != list(range(0, 16384, 37))
    assert all(f(1024, f(1024, p)) == p for p in range(1024))
    assert f(1000, 3) == -1 and f(64, 64) == -1 and f(64, -1) == -1


def test_group_solve_argument_checks_before_touching_a_device():
    import ctypes
    from paper_2203_13283_amd import _lib
    lib = _lib.load()
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    assert lib.cfie_solve_group(None, 0, None, None, None, None, None, 1) == _lib.CFIE_OK
    assert lib.cfie_solve_group(None, -1, None, None, None, None, None, 1) == _lib.CFIE_EINVAL
    assert lib.cfie_solve_group(None, 2, None, None, None, None, None, 1) == _lib.CFIE_EINVAL
    hs = (vp * 1)(None)
    bs = (vp * 1)(None)
    ls = (i64 * 1)(8)
    assert lib.cfie_solve_group(hs, 1, bs, ls, bs, ls, ls, 1) == _lib.CFIE_EINVAL   # NULL ctx
    assert lib.cfie_solve_batch_grouped(None, 0, 1, None, 0, 1) == _lib.CFIE_OK
    assert lib.cfie_solve_batch_grouped(None, 0, 1, None, 0, 0) == _lib.CFIE_EINVAL
    assert lib.cfie_solve_batch_grouped(None, 0, 0, None, 0, 1) == _lib.CFIE_EINVAL


def test_batch_record_reports_disabled_before_touching_a_device():
    """cfie_batch_record is switched off: argument errors still give EINVAL, valid arguments
    EHIP with the reason, with no HIP call and no handle."""
    import ctypes
    from paper_2203_13283_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.cfie_batch_record(None, 0, None, 0, ctypes.byref(h)) == _lib.CFIE_EINVAL
    items = (_lib.BatchItem * 1)()
    items[0].nrhs = 0
    assert lib.cfie_batch_record(None, 0, items, 1, ctypes.byref(h)) == _lib.CFIE_EHIP
    assert b"disabled" in lib.cfie_last_error(None)
    assert not h.value
    assert lib.cfie_batch_nodes(None) == 0
    lib.cfie_batch_destroy(None)


def test_header_is_plain_c(tmp_path):
    """include/cfie.h compiles as ISO C99 with every warning on (a C caller's view)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = tmp_path / "use.c"
    src.write_text('#include "cfie.h"\n'
                   "int main(void) {\n"
                   "    cfie_options o;\n"
                   "    cfie_default_options(&o);\n"
                   "    return (int)cfie_solve_group((cfie_ctx *const *)0, 0, 0, 0, 0, 0, 0, 1);\n"
                   "}\n")
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                        "-fsyntax-only", "-I", os.path.join(root, "include"), str(src)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
