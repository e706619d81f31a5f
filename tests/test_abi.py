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
    # node offsets in the step kernel are 32-bit element counts: nx * ny must
    # stay below 2^32 (field arrays above 4 GiB run the 64-bit-address
    # variant, which is checked on small grids in the GPU tests)
    from paper_1410_0753_amd import clf
    import numpy as np
    x = np.arange(65536.0)
    px = x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    n = ctypes.c_size_t(0)
    lib.clf_workspace_bytes.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    for prec, es in ((clf.FP64, 8), (clf.FP32, 4)):
        p = clf.Params()
        lib.clf_default_params(ctypes.byref(p))
        p.precision = prec
        ok = clf.Grid(65536, 65535, 0, px, px)
        assert lib.clf_workspace_bytes(ctypes.byref(ok), ctypes.byref(p), ctypes.byref(n)) == 0
        assert n.value >= 9 * es * 65536 * 65535
        big = clf.Grid(65536, 65536, 0, px, px)
        assert lib.clf_workspace_bytes(ctypes.byref(big), ctypes.byref(p), ctypes.byref(n)) == -1


def _ws(lib, grid, params):
    import ctypes as C
    n = C.c_size_t(0)
    lib.clf_workspace_bytes.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    return lib.clf_workspace_bytes(C.byref(grid), C.byref(params), C.byref(n))


@pytest.mark.parametrize("field,value", [
    ("precision", 7), ("h_min", 0.0), ("h_min", -1.0), ("manning_n2", -0.1), ("solver", 3),
    ("sweep_order", 5), ("maxout", 0), ("gout", 0), ("bndout", 0), ("ssl_alpha", 0.5),
    ("max_gauges", -1), ("gauge_capacity", -1), ("series_capacity", -1),
    ("earth_radius", 0.0), ("segment", 3), ("segment", 5000), ("graph_steps", 3),
    ("graph_steps", -2), ("persistent_blocks", 12), ("persistent_blocks", -8),
    ("friction_form", 2), ("friction_form", -1), ("open_sides", 16), ("open_sides", -1),
])
def test_parameter_validation(lib, field, value):
    # every parameter outside its documented range is rejected with CLF_EINVAL
    # before anything touches a device
    from paper_1410_0753_amd import clf
    import numpy as np
    x = np.arange(40.0); y = np.arange(30.0)
    px = x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    py = y.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p = clf.Params()
    lib.clf_default_params(ctypes.byref(p))
    g = clf.Grid(40, 30, 0, px, py)
    assert _ws(lib, g, p) == 0
    setattr(p, field, value)
    assert _ws(lib, g, p) == -1


def test_grid_validation(lib):
    from paper_1410_0753_amd import clf
    import numpy as np
    p = clf.Params()
    lib.clf_default_params(ctypes.byref(p))

    def ws(nx, ny, x, y, coord=0):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        g = clf.Grid(nx, ny, coord, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                     y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return _ws(lib, g, p)

    assert ws(3, 3, [0, 1, 2], [0, 1, 2]) == 0
    assert ws(1, 3, [0], [0, 1, 2]) == 0            # 1-D along y
    assert ws(3, 1, [0, 1, 2], [0]) == 0            # 1-D along x
    assert ws(1, 2, [0], [0, 1]) == -1              # 1-D needs 3 nodes
    assert ws(2, 5, [0, 1], np.arange(5)) == -1     # 2-D needs 3 per axis
    assert ws(0, 5, [0], np.arange(5)) == -1
    assert ws(3, 3, [0, 2, 1], [0, 1, 2]) == -1     # x not increasing
    assert ws(3, 3, [0, 1, 2], [0, 1, 1]) == -1     # y not increasing
    assert ws(3, 3, [0, 1, 2], [0, 1, 2], coord=4) == -1
    assert ws(3, 3, [150, 151, 152], [10, 20, 30], coord=1) == 0
    assert ws(3, 3, [150, 151, 152], [80, 85, 90], coord=1) == -1   # latitude out of range
    # the message of a failure without a context is kept for the caller
    lib.clf_last_error.restype = ctypes.c_char_p
    lib.clf_last_error.argtypes = [ctypes.c_void_p]
    assert ws(3, 3, [0, 1, 2], [0, 1, 1]) == -1
    assert b"y not strictly increasing" in lib.clf_last_error(None)


def test_node_index_is_64_bit(lib):
    # gauge node indices iy * nx + ix past 2^31 (grids hold up to 2^32 - 1
    # nodes) round-trip exactly; nodes outside the grid are rejected
    lib.clf_node_index.argtypes = [ctypes.c_int] * 4 + [ctypes.POINTER(ctypes.c_int64)]
    k = ctypes.c_int64(0)
    nx, ny = 65536, 65535
    for ix, iy in ((0, 0), (65535, 32767), (17, 40000), (65535, 65534)):
        assert lib.clf_node_index(nx, ny, ix, iy, ctypes.byref(k)) == 0
        assert k.value == iy * nx + ix
        assert (k.value // nx, k.value % nx) == (iy, ix)
    assert lib.clf_node_index(nx, ny, 65535, 65534, ctypes.byref(k)) == 0 and k.value > 2 ** 32 - 2 ** 17
    for ix, iy in ((-1, 0), (nx, 0), (0, -1), (0, ny)):
        assert lib.clf_node_index(nx, ny, ix, iy, ctypes.byref(k)) == -1
    assert lib.clf_node_index(nx, ny, 0, 0, None) == -1
