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


@pytest.mark.parametrize("n,b", [(22, 4), (40, 6)])
def test_layer_candidates_match_the_slice_partition(n, b):
    # every w >= 2 whose slice subproblems (the oracle's partition along x1 plus
    # b auxiliary lines for every slice after the first) have at most 32 lines
    import numpy as np
    import oracle
    from paper_1705_09443_amd import layer_candidates
    omega = 2 * np.pi * 2.0
    m = np.zeros((n, n))
    alpha, beta, _ = oracle.alpha_beta(oracle.green_table(2, n, omega), n, 2)
    system = oracle.SparseSystem(2, n, omega, m, alpha, beta, b, 10.0)
    expect = []
    for w in range(2, n + 3):
        sw = oracle.Sweep(system, w, m, only=[])
        t = [hi - lo + 1 + (b if k > 0 else 0) for k, (lo, hi) in enumerate(sw.bounds)]
        if max(t) <= 32:
            expect.append(w)
    assert layer_candidates(n, b) == expect


def test_layer_candidates_of_the_full_size_grid_and_bad_arguments():
    # n = 1023, b = 12: 1025 lines; w = 4 leaves a 29-line last slice, w = 6
    # a 35-line one
    from paper_1705_09443_amd import _lib, layer_candidates
    assert layer_candidates(1023, 12) == [2, 3, 4, 5]
    lib = _lib.load()
    cnt = ctypes.c_int()
    assert lib.ls_layer_candidates(0, 12, None, 0, ctypes.byref(cnt)) == _lib.LS_E_INVALID
    assert lib.ls_layer_candidates(63, 12, None, 0, None) == _lib.LS_E_INVALID


def test_setup_without_layer_thickness_needs_autotune():
    # rejected on the host, before any device call
    from paper_1705_09443_amd import _lib
    lib = _lib.load()
    o = _lib.LsOptions()
    lib.ls_default_options(ctypes.byref(o))
    grid = _lib.LsGrid(2, 31)
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)
    assert lib.ls_setup(ctypes.byref(grid), 10.0, dummy, 6, 0, ctypes.byref(o), ctypes.byref(h)) == _lib.LS_E_INVALID
    assert "autotune" in lib.ls_last_error().decode()
    o.autotune = -1
    assert lib.ls_setup(ctypes.byref(grid), 10.0, dummy, 6, 4, ctypes.byref(o), ctypes.byref(h)) == _lib.LS_E_INVALID
    assert not h.value


def test_three_dimensional_grid_passes_the_host_checks():
    # dim = 3 is accepted (Sec. 3.1); these refusals come from the 3D setup's
    # own host checks, before any device call, and name the 3D limits
    from paper_1705_09443_amd import _lib
    lib = _lib.load()
    o = _lib.LsOptions()
    lib.ls_default_options(ctypes.byref(o))
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)
    grid = _lib.LsGrid(3, 2000)
    assert lib.ls_setup(ctypes.byref(grid), 10.0, dummy, 4, 4, ctypes.byref(o), ctypes.byref(h)) == _lib.LS_E_INVALID
    assert "3D: n must be in [1, 1023]" in lib.ls_last_error().decode()
    grid = _lib.LsGrid(3, 15)
    assert lib.ls_setup(ctypes.byref(grid), 10.0, dummy, 4, 0, ctypes.byref(o), ctypes.byref(h)) == _lib.LS_E_INVALID
    assert "3D: layer_thickness" in lib.ls_last_error().decode()
    o.autotune = 4
    assert lib.ls_setup(ctypes.byref(grid), 10.0, dummy, 4, 4, ctypes.byref(o), ctypes.byref(h)) == _lib.LS_E_INVALID
    assert "3D: autotune" in lib.ls_last_error().decode()
    grid = _lib.LsGrid(4, 15)
    o.autotune = 0
    assert lib.ls_setup(ctypes.byref(grid), 10.0, dummy, 4, 4, ctypes.byref(o), ctypes.byref(h)) == _lib.LS_E_INVALID
    assert "dim must be 2 or 3" in lib.ls_last_error().decode()
    assert not h.value


def test_block_size_limits_are_host_checks():
    # block flexible GMRES: groups of at most 64 columns, and the block
    # Hessenberg matrix of a cycle at most 2048 columns wide
    from paper_1705_09443_amd import _lib
    lib = _lib.load()
    o = _lib.LsOptions()
    lib.ls_default_options(ctypes.byref(o))
    assert o.block_size == 1
    grid = _lib.LsGrid(2, 31)
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)
    for bs, rs in ((0, 30), (65, 30), (64, 33)):
        o.block_size, o.restart = bs, rs
        assert lib.ls_setup(ctypes.byref(grid), 10.0, dummy, 6, 4, ctypes.byref(o), ctypes.byref(h)) == \
            _lib.LS_E_INVALID
        assert "block_size" in lib.ls_last_error().decode()
    assert not h.value
