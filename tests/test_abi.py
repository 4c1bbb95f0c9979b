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
    assert lib.cfie_create(None, 0, None, None) == _lib.CFIE_EINVAL
    # NULL context handling of every entry point
    assert lib.cfie_factor(None) == _lib.CFIE_EINVAL
    assert lib.cfie_solve(None, None, 0, None, 0, 0) == _lib.CFIE_EINVAL
    lib.cfie_destroy(None)
