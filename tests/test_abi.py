"""The C-ABI library loads on a host without a GPU and exports every function the header declares;
host-side validation errors come back as status codes without touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2605_07954_amd as lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "mi355stencil.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(lib.LIBPATH):
        from paper_2605_07954_amd import build
        build.build()
    L = ctypes.CDLL(lib.LIBPATH, mode=os.RTLD_NOW)
    names = declared_functions()
    assert len(names) >= 29
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # the Python binding wraps every one of them under the same name
    assert not [n for n in names if n not in ("stencil_strerror", "stencil_last_error") and not hasattr(lib, n)]


def _plan(*a):
    h = ctypes.c_void_p()
    rc = lib.lib().stencil_plan(ctypes.byref(h), *a)
    return rc, h


def test_host_validation_codes():
    W = np.zeros((3, 3), np.float32)
    W[1, 1] = 1
    wp = W.ctypes.data_as(ctypes.c_void_p)
    assert _plan(0, 5, 1, wp, 0.0, 0, 0)[0] == -1           # rows < 1
    assert _plan(5, 5, 0, wp, 0.0, 0, 0)[0] == -1           # radius 0
    assert _plan(5, 5, 5, wp, 0.0, 0, 0)[0] == -1           # radius > 4
    assert _plan(5, 5, 1, None, 0.0, 0, 0)[0] == -1         # NULL weights
    assert _plan(5, 5, 1, wp, float("nan"), 0, 0)[0] == -1  # non-finite b
    assert _plan(5, 5, 1, wp, 0.0, 7, 0)[0] == -1           # unknown storage
    assert _plan(5, 5, 1, wp, 0.0, 0, 0x80)[0] == -1        # unknown flag
    Wn = W.copy()
    Wn[0, 0] = np.inf
    assert _plan(5, 5, 1, Wn.ctypes.data_as(ctypes.c_void_p), 0.0, 0, 0)[0] == -1
    assert "finite" in lib.lib().stencil_last_error().decode()
    rc, h = _plan(5, 5, 1, wp, 0.0, 0, 0)
    assert rc == 0
    try:
        assert lib.stencil_workspace_bytes(h, 0) == 0
        tb, tx, ty = lib.stencil_get_blocking(h)
        lib.stencil_set_blocking(h, 1)
        assert lib.stencil_workspace_bytes(h, 1) == 0
        assert lib.stencil_workspace_bytes(h, 2) == 25 * 4
        with pytest.raises(lib.StencilError):
            lib.stencil_set_blocking(h, 0, 100, 100)   # tile not instantiated
        with pytest.raises(lib.StencilError):
            lib.stencil_set_blocking(h, 17)
    finally:
        lib.stencil_destroy(h)


def test_strerror():
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert lib.lib().stencil_strerror(code)
