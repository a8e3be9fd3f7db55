"""Host-side checks of the C-ABI library (no GPU needed): it loads and exports every symbol that
include/hp.h declares, and the Python binding names the same set."""
import ctypes
import os
import re

import pytest

import paper_1112_3507_amd as hp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "hp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hp_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hp.LIB_PATH):
        from paper_1112_3507_amd import build
        build.build()
    return hp.load_library()


def test_header_declares_binding_exports():
    assert _header_functions() == sorted(hp.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in _header_functions():
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_null_arguments_rejected_without_gpu(lib):
    # argument validation happens before any device call
    out = ctypes.c_void_p()
    assert lib.hp_setup(None, None, None, 1.0, None, ctypes.byref(out)) == hp.EINVAL
    assert b"non-null" in lib.hp_last_error()
    assert lib.hp_solve(None, None, None, 1e-10) == hp.EINVAL
    lib.hp_free(None)
    g = hp.Grid(4, 3, 4, 0.1, 0.1, 0.1)          # odd periodic size
    b = hp.BC(hp.PERIODIC, hp.PERIODIC, hp.NEUMANN)
    fake = ctypes.c_void_p(16)
    assert lib.hp_setup(ctypes.byref(g), fake, fake, 1.0, ctypes.byref(b), ctypes.byref(out)) == hp.EINVAL
    assert b"even" in lib.hp_last_error()
    g = hp.Grid(4, 4, 4, 0.1, 0.1, 0.1)
    assert lib.hp_setup(ctypes.byref(g), fake, fake, -1.0, ctypes.byref(b), ctypes.byref(out)) == hp.EINVAL
    assert lib.hp_set_option(None, hp.OPT_MODE, 1.0) == hp.EINVAL
