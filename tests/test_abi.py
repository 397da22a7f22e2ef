"""The C-ABI library loads and exports every entry point include/lsweep.h
declares (no device needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "lsweep.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ls_[A-Za-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    from paper_1705_09443_amd import _lib
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 17
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib._SIGNATURES, f"{name} has no binding"


def test_library_is_built_for_gfx950():
    from paper_1705_09443_amd import _lib
    _lib.load()
    data = open(_lib.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_default_options_and_error_channel():
    from paper_1705_09443_amd import _lib
    lib = _lib.load()
    o = _lib.LsOptions()
    lib.ls_default_options(ctypes.byref(o))
    assert (o.precision, o.restart, o.max_iters, o.pml_C) == (0, 30, 1000, 10.0)
    # invalid argument is reported without touching a device
    st = lib.ls_setup(None, 1.0, None, 12, 4, None, None)
    assert st == _lib.LS_E_INVALID
    assert lib.ls_last_error().decode()
    lib.ls_destroy(None)  # no-op
