"""The C-ABI library loads and exports every function include/clf.h declares
(no GPU needed: nothing is called that touches a device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "clf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(clf_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1410_0753_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    return ctypes.CDLL(build.LIB)


def test_header_declares_the_binding_list():
    from paper_1410_0753_amd import clf
    assert declared_functions() == sorted(clf.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_default_params_and_workspace_size(lib):
    from paper_1410_0753_amd import clf
    p = clf.Params()
    lib.clf_default_params(ctypes.byref(p))
    assert p.solver == 2 and p.ssl_alpha == 2.0 and abs(p.h_min - 0.1) < 1e-15
    import numpy as np
    x = np.arange(100.0); y = np.arange(50.0)
    g = clf.Grid(100, 50, 0, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                 y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    n = ctypes.c_size_t(0)
    lib.clf_workspace_bytes.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.clf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(n)) == 0
    assert n.value >= 9 * 8 * 100 * 50
    bad = clf.Grid(2, 50, 0, g.x, g.y)
    assert lib.clf_workspace_bytes(ctypes.byref(bad), ctypes.byref(p), ctypes.byref(n)) == -1


def test_grid_size_limits(lib):
    # the step kernel uses 32-bit element offsets: nx * ny must stay below 2^32
    from paper_1410_0753_amd import clf
    import numpy as np
    p = clf.Params()
    lib.clf_default_params(ctypes.byref(p))
    x = np.arange(65536.0)
    px = x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    n = ctypes.c_size_t(0)
    lib.clf_workspace_bytes.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    big = clf.Grid(65536, 65536, 0, px, px)
    assert lib.clf_workspace_bytes(ctypes.byref(big), ctypes.byref(p), ctypes.byref(n)) == -1
    ok = clf.Grid(65536, 65535, 0, px, px)
    assert lib.clf_workspace_bytes(ctypes.byref(ok), ctypes.byref(p), ctypes.byref(n)) == 0
    assert n.value >= 9 * 8 * 65536 * 65535
