"""Python wrapper of the FP64 CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It compiles ``cliffs_oracle.cpp`` with
g++ on demand (``-O2 -ffp-contract=off -fopenmp``) and drives it through
ctypes on host numpy arrays.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cliffs_oracle.cpp")
_LIB = os.path.join(_HERE, "_build", "libcliffs_oracle.so")
# A prebuilt copy of the oracle to load instead (used by the mutation tests,
# which compile the oracle with one planted mistake and expect a pin to fail).
_LIB_OVERRIDE = os.environ.get("CLF_ORACLE_LIB")
_lock = threading.Lock()
_lib = None

CARTESIAN, SPHERICAL = 0, 1
ORDER_XY, ORDER_ALTERNATE = 0, 1
FRICTION_EXPLICIT, FRICTION_SEMI_IMPLICIT = 0, 1
OPEN_W, OPEN_E, OPEN_S, OPEN_N = 1, 2, 4, 8
G = 9.81
R_EARTH = 6371000.0

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_up = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the oracle library if missing or older than its source."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c++17",
               "-shared", "-fPIC", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            L = C.CDLL(_LIB_OVERRIDE or build())
            L.ora_create.restype = C.c_void_p
            L.ora_create.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, C.c_double,
                                     C.c_double, C.c_double, C.c_int, C.c_double, C.c_double,
                                     C.c_double, C.c_int, C.c_int, C.c_double, C.c_int,
                                     C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                     C.POINTER(C.c_int)]
            L.ora_destroy.argtypes = [C.c_void_p]
            L.ora_set_threads.argtypes = [C.c_int]
            L.ora_cs_record_loss.argtypes = [C.c_void_p] + [_dp] * 6 + [
                C.c_double, C.c_int, _dp, _dp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
            L.ora_ssl_passes.argtypes = [C.c_void_p]
            L.ora_max_cfl.argtypes = [C.c_void_p]
            L.ora_max_cfl.restype = C.c_double
            L.ora_get_depth.argtypes = [C.c_void_p, _dp]
            L.ora_set_initial.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
            L.ora_set_raw_state.argtypes = [C.c_void_p, _dp, _dp, _dp, C.c_long]
            L.ora_get_raw_state.argtypes = [C.c_void_p, _dp, _dp, _dp]
            L.ora_get_state.argtypes = [C.c_void_p, _dp, _dp, _dp, _up]
            L.ora_step_count.argtypes = [C.c_void_p]
            L.ora_step_count.restype = C.c_long
            L.ora_step.argtypes = [C.c_void_p, C.c_int]
            L.ora_sweep.argtypes = [C.c_void_p, C.c_int]
            L.ora_set_gauges.argtypes = [C.c_void_p, C.c_int, _ip, _ip]
            L.ora_num_gauge_records.argtypes = [C.c_void_p]
            L.ora_read_gauges.argtypes = [C.c_void_p, _dp, _dp]
            L.ora_read_maxwave.argtypes = [C.c_void_p, _dp, _dp]
            L.ora_add_enclosed.argtypes = [C.c_void_p, C.c_int, C.c_int, _dp, _dp]
            L.ora_num_series_records.argtypes = [C.c_void_p, C.c_int]
            L.ora_read_series.argtypes = [C.c_void_p, C.c_int, C.c_int, _dp, _dp]
            L.ora_set_forcing.argtypes = [C.c_void_p, C.c_int, C.c_int, _dp, _dp]
            L.ora_ssl.argtypes = [C.c_int, C.c_int, _dp, C.c_double, C.c_double]
            L.ora_cs_gauge_loss.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_int, _dp,
                                            C.POINTER(C.c_double), C.POINTER(C.c_double)]
            _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def ssl(depth, alpha=2.0, min_depth=0.1):
    """Depth preprocessing on a copy; returns (new depth, passes)."""
    d = _f64(depth).copy()
    ny, nx = d.shape
    passes = lib().ora_ssl(nx, ny, d, alpha, min_depth)
    return d, passes


def set_threads(n: int) -> int:
    """Thread count of the oracle's row / column loops (n <= 0: OpenMP
    default); returns the count in use.  Results do not depend on it."""
    return int(lib().ora_set_threads(int(n)))


class Oracle:
    """Oracle model: the same semantic calls as the GPU library, on host arrays."""

    def __init__(self, x, y, depth, dt, coord=CARTESIAN, h_min=0.1, manning_n2=0.0,
                 itopo=1, dwall=0.0, ssl_alpha=2.0, ssl_min_depth=0.1, order=ORDER_XY,
                 solver=2, earth_radius=R_EARTH, spherical_metric=1, maxout=1, gout=1,
                 bndout=1, sweep_order=None, friction_form=0, open_sides=0, **device_only):
        # capacities and limits of the GPU library have no meaning here
        unknown = set(device_only) - {"precision", "cfl_limit", "max_gauges", "gauge_capacity",
                                      "max_enclosed", "max_enclosed_points", "series_capacity",
                                      "forcing_capacity"}
        if unknown:
            raise TypeError("unknown oracle parameter(s) %s" % sorted(unknown))
        if sweep_order is not None:
            order = sweep_order
        L = lib()
        depth = _f64(depth)
        self.ny, self.nx = depth.shape
        self.x, self.y = _f64(x), _f64(y)
        st = C.c_int(0)
        self._h = L.ora_create(self.nx, self.ny, coord, self.x, self.y, depth, dt, h_min,
                               manning_n2, itopo, dwall, ssl_alpha, ssl_min_depth, order, solver,
                               earth_radius, spherical_metric, maxout, gout, bndout,
                               int(friction_form), int(open_sides), C.byref(st))
        if not self._h:
            raise ValueError("oracle init failed (status %d)" % st.value)
        self.dt = dt
        self.h_min = h_min
        self._keep = []

    @classmethod
    def from_case(cls, case, **kw):
        kw.setdefault("h_min", case.h_min)
        kw.setdefault("manning_n2", getattr(case, "manning_n2", 0.0))
        kw.setdefault("friction_form", getattr(case, "friction_form", 0))
        return cls(case.x, case.y, case.depth, case.dt, coord=case.coord, **kw)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().ora_destroy(h)
            self._h = None

    # -- setup --
    @property
    def ssl_passes(self):
        return lib().ora_ssl_passes(self._h)

    def max_cfl(self):
        return lib().ora_max_cfl(self._h)

    def depth(self):
        d = np.empty((self.ny, self.nx))
        lib().ora_get_depth(self._h, d)
        return d

    def set_initial(self, eta=None, u=None, v=None, deform_bottom=False):
        arrs = [None if a is None else _f64(a).reshape(self.ny, self.nx) for a in (eta, u, v)]
        lib().ora_set_initial(self._h, *[_ptr(a) for a in arrs], int(bool(deform_bottom)))

    def set_raw_state(self, H, u, v, n):
        lib().ora_set_raw_state(self._h, _f64(H), _f64(u), _f64(v), int(n))

    def raw_state(self):
        H, u, v = (np.empty((self.ny, self.nx)) for _ in range(3))
        lib().ora_get_raw_state(self._h, H, u, v)
        return H, u, v

    def state(self):
        e, u, v = (np.empty((self.ny, self.nx)) for _ in range(3))
        w = np.empty((self.ny, self.nx), dtype=np.uint8)
        lib().ora_get_state(self._h, e, u, v, w)
        return e, u, v, w

    @property
    def n(self):
        return lib().ora_step_count(self._h)

    def step(self, n=1):
        lib().ora_step(self._h, int(n))

    def sweep(self, axis):
        lib().ora_sweep(self._h, int(axis))

    def set_gauges(self, ix, iy):
        ix = np.ascontiguousarray(ix, dtype=np.int32)
        iy = np.ascontiguousarray(iy, dtype=np.int32)
        if lib().ora_set_gauges(self._h, len(ix), ix, iy) != 0:
            raise ValueError("bad gauge index")
        self._ng = len(ix)

    def read_gauges(self):
        n = lib().ora_num_gauge_records(self._h)
        out = np.empty((n, self._ng, 3))
        t = np.empty(n)
        lib().ora_read_gauges(self._h, out, t)
        return out, t

    def read_maxwave(self):
        e, s = np.empty((self.ny, self.nx)), np.empty((self.ny, self.nx))
        lib().ora_read_maxwave(self._h, e, s)
        return e, s

    def add_enclosed_grid(self, x, y):
        x, y = _f64(x), _f64(y)
        gid = lib().ora_add_enclosed(self._h, len(x), len(y), x, y)
        if gid < 0:
            raise ValueError("enclosed grid outside the master grid")
        if not hasattr(self, "_enc"):
            self._enc = []
        self._enc.append((len(x), len(y)))
        return gid

    def read_boundary_series(self, gid, side):
        nxe, nye = self._enc[gid]
        np_ = nye if side < 2 else nxe
        n = lib().ora_num_series_records(self._h, gid)
        vals = np.empty((n, 3, np_))
        t = np.empty(n)
        lib().ora_read_series(self._h, gid, side, vals, t)
        return vals, t

    def set_boundary_forcing(self, side, t, vals):
        t, vals = _f64(t), _f64(vals)
        if lib().ora_set_forcing(self._h, side, len(t), t, vals) != 0:
            raise ValueError("bad forcing")

    def cs_record_loss(self, eta0, u0, v0, deta, du, dv, nsteps, obs, w=(1.0, 1.0, 1.0),
                       h=1e-30):
        """Weighted misfit of all gauge records (eta, u, v) and its complex-step
        derivative along (deta, du, dv) of the initial state."""
        L, dL = C.c_double(0), C.c_double(0)
        lib().ora_cs_record_loss(self._h, _f64(eta0), _f64(u0), _f64(v0), _f64(deta), _f64(du),
                                 _f64(dv), h, int(nsteps), _f64(obs), _f64(np.asarray(w)),
                                 C.byref(L), C.byref(dL))
        return L.value, dL.value

    def cs_gauge_loss(self, eta0, deta, nsteps, obs, h=1e-30):
        L, dL = C.c_double(0), C.c_double(0)
        lib().ora_cs_gauge_loss(self._h, _f64(eta0), _f64(deta), h, int(nsteps), _f64(obs),
                                C.byref(L), C.byref(dL))
        return L.value, dL.value
