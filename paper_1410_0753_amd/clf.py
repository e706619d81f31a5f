"""ctypes binding of libclf.so (argument marshalling only).

Every computation runs in the HIP library; this module converts torch
tensors / numpy arrays to pointers, keeps the caller-owned workspace alive
and raises on non-zero return codes.  There is no CPU fallback: without the
built library or a GPU the calls fail.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libclf.so")

CLF_OK = 0
ERRORS = {-1: "CLF_EINVAL", -2: "CLF_ECFL", -3: "CLF_EHIP", -4: "CLF_ENONFINITE",
          -5: "CLF_ESTATE", -6: "CLF_ENOSPACE", -7: "CLF_ESSL"}
CARTESIAN, SPHERICAL = 0, 1
FP64, FP32 = 0, 1
ORDER_XY, ORDER_ALTERNATE = 0, 1
WEST, EAST, SOUTH, NORTH = 0, 1, 2, 3
FRICTION_EXPLICIT, FRICTION_SEMI_IMPLICIT = 0, 1
OPEN_W, OPEN_E, OPEN_S, OPEN_N = 1, 2, 4, 8
(Q_MAX_CFL, Q_SSL_PASSES, Q_STEP, Q_MIN_F, Q_WORKSPACE, Q_GAUGE_RECORDS, Q_TILES, Q_SEGMENT,
 Q_BLOCKS, Q_GRAPH_REPLAYS, Q_WIDE, Q_KERNEL_MS, Q_KERNEL_LAUNCHES, Q_KERNEL_RESET,
 Q_LDS_ROWS) = range(1, 16)

# Every symbol include/clf.h declares.
EXPORTS = ["clf_default_params", "clf_node_index", "clf_workspace_bytes", "clf_init", "clf_set_initial",
           "clf_set_raw_state", "clf_get_raw_state", "clf_set_boundary_forcing", "clf_set_gauges",
           "clf_add_enclosed_grid", "clf_step", "clf_sweep", "clf_get_state", "clf_get_depth",
           "clf_read_gauges", "clf_read_maxwave", "clf_read_boundary_series",
           "clf_clear_records", "clf_sync", "clf_query", "clf_last_error", "clf_destroy",
           "clf_ensemble_workspace_bytes", "clf_ensemble_init", "clf_ensemble_set_initial",
           "clf_ensemble_step", "clf_ensemble_get_state", "clf_ensemble_read_maxwave",
           "clf_ensemble_sync", "clf_ensemble_query", "clf_ensemble_last_error",
           "clf_ensemble_destroy", "clf_adjoint_workspace_bytes", "clf_adjoint_forward",
           "clf_adjoint_backward", "clf_step_static", "clf_bands_workspace_bytes",
           "clf_bands_init", "clf_bands_set_initial", "clf_bands_step", "clf_bands_get_state",
           "clf_bands_read_maxwave", "clf_bands_sync", "clf_bands_query",
           "clf_bands_last_error", "clf_bands_destroy"]


class ClfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("coord", C.c_int32),
                ("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double))]


class Params(C.Structure):
    _fields_ = [("precision", C.c_int32), ("h_min", C.c_double), ("manning_n2", C.c_double),
                ("itopo", C.c_int32), ("dwall", C.c_double), ("ssl_alpha", C.c_double),
                ("ssl_min_depth", C.c_double), ("sweep_order", C.c_int32), ("solver", C.c_int32),
                ("earth_radius", C.c_double), ("spherical_metric", C.c_int32),
                ("cfl_limit", C.c_double), ("maxout", C.c_int32), ("gout", C.c_int32),
                ("bndout", C.c_int32), ("max_gauges", C.c_int32), ("gauge_capacity", C.c_int32),
                ("max_enclosed", C.c_int32), ("max_enclosed_points", C.c_int32),
                ("series_capacity", C.c_int32), ("forcing_capacity", C.c_int32),
                ("segment", C.c_int32), ("autotune", C.c_int32),
                ("graph_steps", C.c_int32), ("persistent_blocks", C.c_int32),
                ("friction_form", C.c_int32), ("open_sides", C.c_int32),
                ("kernel_timing", C.c_int32)]


_lock = threading.Lock()
_lib = None


def load(build_if_missing: bool = True):
    """Load libclf.so (building it with hipcc first if it is absent)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            if not build_if_missing:
                raise RuntimeError("libclf.so is not built")
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        vp, i32, dbl = C.c_void_p, C.c_int, C.c_double
        sig = {
            "clf_default_params": (None, [C.POINTER(Params)]),
            "clf_node_index": (i32, [i32, i32, i32, i32, C.POINTER(C.c_int64)]),
            "clf_workspace_bytes": (i32, [C.POINTER(Grid), C.POINTER(Params), C.POINTER(C.c_size_t)]),
            "clf_init": (i32, [C.POINTER(vp), C.POINTER(Grid), vp, dbl, C.POINTER(Params), vp, vp,
                               C.c_size_t]),
            "clf_set_initial": (i32, [vp, vp, vp, vp, i32]),
            "clf_set_raw_state": (i32, [vp, vp, vp, vp, C.c_int64]),
            "clf_get_raw_state": (i32, [vp, vp, vp, vp]),
            "clf_set_boundary_forcing": (i32, [vp, i32, i32, vp, vp]),
            "clf_set_gauges": (i32, [vp, i32, vp, vp]),
            "clf_add_enclosed_grid": (i32, [vp, i32, i32, vp, vp, C.POINTER(i32)]),
            "clf_step": (i32, [vp, i32]),
            "clf_sweep": (i32, [vp, i32]),
            "clf_get_state": (i32, [vp, vp, vp, vp, vp]),
            "clf_get_depth": (i32, [vp, vp]),
            "clf_read_gauges": (i32, [vp, vp, vp, C.POINTER(i32), i32]),
            "clf_read_maxwave": (i32, [vp, vp, vp]),
            "clf_read_boundary_series": (i32, [vp, i32, i32, vp, vp, C.POINTER(i32), i32]),
            "clf_clear_records": (i32, [vp]),
            "clf_sync": (i32, [vp]),
            "clf_query": (i32, [vp, i32, C.POINTER(dbl)]),
            "clf_last_error": (C.c_char_p, [vp]),
            "clf_destroy": (i32, [vp]),
            "clf_ensemble_workspace_bytes": (i32, [i32, vp, C.POINTER(Params), C.POINTER(C.c_size_t)]),
            "clf_ensemble_init": (i32, [C.POINTER(vp), i32, vp, vp, vp, C.POINTER(Params), vp, vp,
                                        C.c_size_t]),
            "clf_ensemble_set_initial": (i32, [vp, i32, vp, vp, vp, i32]),
            "clf_ensemble_step": (i32, [vp, i32]),
            "clf_ensemble_get_state": (i32, [vp, i32, vp, vp, vp, vp]),
            "clf_ensemble_read_maxwave": (i32, [vp, i32, vp, vp]),
            "clf_ensemble_sync": (i32, [vp]),
            "clf_ensemble_query": (i32, [vp, i32, C.POINTER(dbl)]),
            "clf_ensemble_last_error": (C.c_char_p, [vp]),
            "clf_ensemble_destroy": (i32, [vp]),
            "clf_adjoint_workspace_bytes": (i32, [vp, i32, i32, C.POINTER(C.c_size_t)]),
            "clf_adjoint_forward": (i32, [vp, i32, i32, vp, C.c_size_t]),
            "clf_adjoint_backward": (i32, [vp, vp, i32, vp, vp, vp]),
            "clf_step_static": (i32, [C.POINTER(Grid), C.POINTER(Params), dbl, vp, vp, vp, vp,
                                      vp, vp, vp, vp, vp, i32, vp, C.POINTER(i32)]),
            "clf_bands_workspace_bytes": (i32, [C.POINTER(Grid), C.POINTER(Params), i32,
                                                C.POINTER(C.c_size_t)]),
            "clf_bands_init": (i32, [C.POINTER(vp), C.POINTER(Grid), vp, dbl, C.POINTER(Params),
                                     i32, vp, vp, C.c_size_t]),
            "clf_bands_set_initial": (i32, [vp, vp, vp, vp, i32]),
            "clf_bands_step": (i32, [vp, i32]),
            "clf_bands_get_state": (i32, [vp, vp, vp, vp, vp]),
            "clf_bands_read_maxwave": (i32, [vp, vp, vp]),
            "clf_bands_sync": (i32, [vp]),
            "clf_bands_query": (i32, [vp, i32, C.POINTER(dbl)]),
            "clf_bands_last_error": (C.c_char_p, [vp]),
            "clf_bands_destroy": (i32, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        return L


def default_params(**kw) -> Params:
    p = Params()
    load().clf_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError("unknown parameter %r" % k)
        setattr(p, k, v)
    return p


def _np64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


class Solver:
    """One grid: the C-ABI context plus its torch-owned workspace."""

    def __init__(self, x, y, depth, dt, coord=CARTESIAN, precision=FP64, device=None,
                 stream=None, **params):
        import torch
        self.torch = torch
        L = load()
        self.device = torch.device(device or "cuda")
        depth = _np64(depth)
        self.ny, self.nx = depth.shape
        self._x, self._y = _np64(x), _np64(y)
        if self._x.shape != (self.nx,) or self._y.shape != (self.ny,):
            raise ValueError("coordinate lengths do not match the depth array")
        self.grid = Grid(self.nx, self.ny, coord,
                         self._x.ctypes.data_as(C.POINTER(C.c_double)),
                         self._y.ctypes.data_as(C.POINTER(C.c_double)))
        self.params = default_params(precision=precision, **params)
        nbytes = C.c_size_t(0)
        self._check_init(L.clf_workspace_bytes(C.byref(self.grid), C.byref(self.params),
                                               C.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        self._check_init(L.clf_init(C.byref(h), C.byref(self.grid),
                                    depth.ctypes.data_as(C.c_void_p), float(dt),
                                    C.byref(self.params), C.c_void_p(self.stream.cuda_stream),
                                    C.c_void_p(self.workspace.data_ptr()), nbytes.value))
        self._h = h
        self.dt = float(dt)
        self.coord = coord
        self.precision = precision
        self._ng = 0
        self._enc = []

    @classmethod
    def from_case(cls, case, **kw):
        kw.setdefault("h_min", case.h_min)
        kw.setdefault("manning_n2", getattr(case, "manning_n2", 0.0))
        kw.setdefault("friction_form", getattr(case, "friction_form", 0))
        return cls(case.x, case.y, case.depth, case.dt, coord=case.coord, **kw)

    # -- errors --
    def _check_init(self, rc):
        if rc != CLF_OK:
            raise ClfError(rc, load().clf_last_error(None).decode())

    def _check(self, rc):
        if rc != CLF_OK:
            raise ClfError(rc, load().clf_last_error(self._h).decode())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.clf_destroy(h)
            self._h = None

    # -- helpers --
    def _dev64(self, a):
        if a is None:
            return None
        t = self.torch
        if isinstance(a, t.Tensor):
            a = a.to(device=self.device, dtype=t.float64)
        else:
            a = t.from_numpy(_np64(a)).to(self.device)
        a = a.reshape(self.ny, self.nx).contiguous()
        return a

    def _empty(self, dtype=None):
        t = self.torch
        return t.empty((self.ny, self.nx), dtype=dtype or t.float64, device=self.device)

    # -- calls --
    def set_initial(self, eta=None, u=None, v=None, deform_bottom=False):
        e, uu, vv = (self._dev64(a) for a in (eta, u, v))
        self._check(load().clf_set_initial(self._h, _dptr(e), _dptr(uu), _dptr(vv),
                                           int(bool(deform_bottom))))
        self.torch.cuda.synchronize(self.device)

    def set_raw_state(self, h, u, v, n):
        hh, uu, vv = (self._dev64(a) for a in (h, u, v))
        self._check(load().clf_set_raw_state(self._h, _dptr(hh), _dptr(uu), _dptr(vv), int(n)))
        self.torch.cuda.synchronize(self.device)

    def raw_state(self):
        h, u, v = self._empty(), self._empty(), self._empty()
        self._check(load().clf_get_raw_state(self._h, _dptr(h), _dptr(u), _dptr(v)))
        return h, u, v

    def state(self):
        t = self.torch
        e, u, v = self._empty(), self._empty(), self._empty()
        w = self._empty(t.uint8)
        self._check(load().clf_get_state(self._h, _dptr(e), _dptr(u), _dptr(v), _dptr(w)))
        return e, u, v, w

    def depth(self):
        d = self._empty()
        self._check(load().clf_get_depth(self._h, _dptr(d)))
        return d

    def step(self, n=1):
        self._check(load().clf_step(self._h, int(n)))

    def sweep(self, axis):
        self._check(load().clf_sweep(self._h, int(axis)))

    def sync(self):
        self._check(load().clf_sync(self._h))

    def set_gauges(self, ix, iy):
        ix = np.ascontiguousarray(ix, dtype=np.int32)
        iy = np.ascontiguousarray(iy, dtype=np.int32)
        self._check(load().clf_set_gauges(self._h, len(ix), ix.ctypes.data_as(C.c_void_p),
                                          iy.ctypes.data_as(C.c_void_p)))
        self._ng = len(ix)

    def read_gauges(self):
        n = C.c_int(0)
        self._check(load().clf_read_gauges(self._h, None, None, C.byref(n), 0))
        out = np.empty((n.value, self._ng, 3))
        times = np.empty(n.value)
        self._check(load().clf_read_gauges(self._h, out.ctypes.data_as(C.c_void_p),
                                           times.ctypes.data_as(C.c_void_p), C.byref(n), n.value))
        return out, times

    def read_maxwave(self):
        e, s = self._empty(), self._empty()
        self._check(load().clf_read_maxwave(self._h, _dptr(e), _dptr(s)))
        return e, s

    def add_enclosed_grid(self, x, y):
        x, y = _np64(x), _np64(y)
        gid = C.c_int(-1)
        self._check(load().clf_add_enclosed_grid(self._h, len(x), len(y),
                                                 x.ctypes.data_as(C.c_void_p),
                                                 y.ctypes.data_as(C.c_void_p), C.byref(gid)))
        self._enc.append((len(x), len(y)))
        return gid.value

    def read_boundary_series(self, gid, side):
        nxe, nye = self._enc[gid]
        np_ = nye if side < 2 else nxe
        n = C.c_int(0)
        self._check(load().clf_read_boundary_series(self._h, gid, side, None, None, C.byref(n), 0))
        vals = np.empty((n.value, 3, np_))
        times = np.empty(n.value)
        self._check(load().clf_read_boundary_series(self._h, gid, side,
                                                    vals.ctypes.data_as(C.c_void_p),
                                                    times.ctypes.data_as(C.c_void_p), C.byref(n),
                                                    n.value))
        return vals, times

    def clear_records(self):
        self._check(load().clf_clear_records(self._h))

    def set_boundary_forcing(self, side, t, vals):
        t, vals = _np64(t), _np64(vals)
        self._check(load().clf_set_boundary_forcing(self._h, int(side), len(t),
                                                    t.ctypes.data_as(C.c_void_p),
                                                    vals.ctypes.data_as(C.c_void_p)))

    def query(self, what):
        v = C.c_double(0)
        self._check(load().clf_query(self._h, int(what), C.byref(v)))
        return v.value

    # -- adjoint --
    def adjoint_forward(self, nsteps, ckpt_every=0):
        """Forward run of nsteps from clf_set_initial, keeping checkpoints.
        Each call replaces the previous run's checkpoints and counts up
        `adjoint_generation`."""
        nb = C.c_size_t(0)
        self._check(load().clf_adjoint_workspace_bytes(self._h, int(nsteps), int(ckpt_every),
                                                       C.byref(nb)))
        self.adj_workspace = self.torch.empty(int(nb.value), dtype=self.torch.uint8,
                                              device=self.device)
        self.adjoint_generation = getattr(self, "adjoint_generation", 0) + 1
        self._check(load().clf_adjoint_forward(self._h, int(nsteps), int(ckpt_every),
                                               C.c_void_p(self.adj_workspace.data_ptr()),
                                               nb.value))

    def adjoint_backward(self, rec_adj):
        """rec_adj [nrec][ng][3] -> (dL/deta0, dL/du0, dL/dv0) device tensors."""
        r = np.ascontiguousarray(rec_adj, dtype=np.float64)
        de, du, dv = self._empty(), self._empty(), self._empty()
        self._check(load().clf_adjoint_backward(self._h, r.ctypes.data_as(C.c_void_p), r.shape[0],
                                                _dptr(de), _dptr(du), _dptr(dv)))
        return de, du, dv


class Ensemble:
    """Many grids advanced in lockstep by one step-kernel launch per step."""

    def __init__(self, cases, precision=FP64, device=None, stream=None, **params):
        import torch
        self.torch = torch
        L = load()
        self.device = torch.device(device or "cuda")
        n = len(cases)
        self._keep = []
        grids = (Grid * n)()
        depths = (C.c_void_p * n)()
        dts = (C.c_double * n)()
        self.shapes = []
        for i, cs in enumerate(cases):
            x, y, d = _np64(cs.x), _np64(cs.y), _np64(cs.depth)
            self._keep += [x, y, d]
            grids[i] = Grid(d.shape[1], d.shape[0], cs.coord, x.ctypes.data_as(C.POINTER(C.c_double)),
                            y.ctypes.data_as(C.POINTER(C.c_double)))
            depths[i] = d.ctypes.data_as(C.c_void_p)
            dts[i] = float(cs.dt)
            self.shapes.append(d.shape)
        params.setdefault("h_min", cases[0].h_min)
        self.params = default_params(precision=precision, **params)
        nbytes = C.c_size_t(0)
        rc = L.clf_ensemble_workspace_bytes(n, grids, C.byref(self.params), C.byref(nbytes))
        self._chk(rc, None)
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = L.clf_ensemble_init(C.byref(h), n, grids, depths, dts, C.byref(self.params),
                                 C.c_void_p(self.stream.cuda_stream),
                                 C.c_void_p(self.workspace.data_ptr()), nbytes.value)
        self._chk(rc, None)
        self._h = h
        self.n = n

    def _chk(self, rc, h):
        if rc != CLF_OK:
            raise ClfError(rc, load().clf_ensemble_last_error(h).decode())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.clf_ensemble_destroy(h)
            self._h = None

    def _dev64(self, a, shape):
        if a is None:
            return None
        t = self.torch
        if isinstance(a, t.Tensor):
            a = a.to(device=self.device, dtype=t.float64)
        else:
            a = t.from_numpy(_np64(a)).to(self.device)
        return a.reshape(shape).contiguous()

    def set_initial(self, member, eta=None, u=None, v=None, deform_bottom=False):
        sh = self.shapes[member]
        e, uu, vv = (self._dev64(a, sh) for a in (eta, u, v))
        self._chk(load().clf_ensemble_set_initial(self._h, member, _dptr(e), _dptr(uu), _dptr(vv),
                                                  int(bool(deform_bottom))), self._h)
        self.torch.cuda.synchronize(self.device)

    def step(self, n=1):
        self._chk(load().clf_ensemble_step(self._h, int(n)), self._h)

    def sync(self):
        self._chk(load().clf_ensemble_sync(self._h), self._h)

    def state(self, member):
        t = self.torch
        sh = self.shapes[member]
        e, u, v = (t.empty(sh, dtype=t.float64, device=self.device) for _ in range(3))
        w = t.empty(sh, dtype=t.uint8, device=self.device)
        self._chk(load().clf_ensemble_get_state(self._h, member, _dptr(e), _dptr(u), _dptr(v),
                                                _dptr(w)), self._h)
        return e, u, v, w

    def read_maxwave(self, member):
        t = self.torch
        sh = self.shapes[member]
        e, s = (t.empty(sh, dtype=t.float64, device=self.device) for _ in range(2))
        self._chk(load().clf_ensemble_read_maxwave(self._h, member, _dptr(e), _dptr(s)), self._h)
        return e, s

    def query(self, what):
        v = C.c_double(0)
        self._chk(load().clf_ensemble_query(self._h, int(what), C.byref(v)), self._h)
        return v.value


class Bands:
    """One grid split into y-bands on one device (whole-grid arrays in and
    out; the band layout stays inside the library)."""

    def __init__(self, x, y, depth, dt, nbands, coord=CARTESIAN, precision=FP64, device=None,
                 stream=None, **params):
        import torch
        self.torch = torch
        L = load()
        self.device = torch.device(device or "cuda")
        depth = _np64(depth)
        self.ny, self.nx = depth.shape
        self._x, self._y = _np64(x), _np64(y)
        self.grid = Grid(self.nx, self.ny, coord,
                         self._x.ctypes.data_as(C.POINTER(C.c_double)),
                         self._y.ctypes.data_as(C.POINTER(C.c_double)))
        self.params = default_params(precision=precision, **params)
        nbytes = C.c_size_t(0)
        self._chk(L.clf_bands_workspace_bytes(C.byref(self.grid), C.byref(self.params),
                                              int(nbands), C.byref(nbytes)), None)
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        self._chk(L.clf_bands_init(C.byref(h), C.byref(self.grid),
                                   depth.ctypes.data_as(C.c_void_p), float(dt),
                                   C.byref(self.params), int(nbands),
                                   C.c_void_p(self.stream.cuda_stream),
                                   C.c_void_p(self.workspace.data_ptr()), nbytes.value), None)
        self._h = h

    @classmethod
    def from_case(cls, case, nbands, **kw):
        kw.setdefault("h_min", case.h_min)
        kw.setdefault("manning_n2", getattr(case, "manning_n2", 0.0))
        kw.setdefault("friction_form", getattr(case, "friction_form", 0))
        return cls(case.x, case.y, case.depth, case.dt, nbands, coord=case.coord, **kw)

    def _chk(self, rc, h):
        if rc != CLF_OK:
            raise ClfError(rc, load().clf_bands_last_error(h).decode())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.clf_bands_destroy(h)
            self._h = None

    def _dev64(self, a):
        if a is None:
            return None
        t = self.torch
        if isinstance(a, t.Tensor):
            a = a.to(device=self.device, dtype=t.float64)
        else:
            a = t.from_numpy(_np64(a)).to(self.device)
        return a.reshape(self.ny, self.nx).contiguous()

    def set_initial(self, eta=None, u=None, v=None, deform_bottom=False):
        e, uu, vv = (self._dev64(a) for a in (eta, u, v))
        self._chk(load().clf_bands_set_initial(self._h, _dptr(e), _dptr(uu), _dptr(vv),
                                               int(bool(deform_bottom))), self._h)
        self.torch.cuda.synchronize(self.device)

    def step(self, n=1):
        self._chk(load().clf_bands_step(self._h, int(n)), self._h)

    def sync(self):
        self._chk(load().clf_bands_sync(self._h), self._h)

    def state(self):
        t = self.torch
        e, u, v = (t.empty((self.ny, self.nx), dtype=t.float64, device=self.device)
                   for _ in range(3))
        w = t.empty((self.ny, self.nx), dtype=t.uint8, device=self.device)
        self._chk(load().clf_bands_get_state(self._h, _dptr(e), _dptr(u), _dptr(v), _dptr(w)),
                  self._h)
        return e, u, v, w

    def read_maxwave(self):
        t = self.torch
        e, s = (t.empty((self.ny, self.nx), dtype=t.float64, device=self.device)
                for _ in range(2))
        self._chk(load().clf_bands_read_maxwave(self._h, _dptr(e), _dptr(s)), self._h)
        return e, s

    def query(self, what):
        v = C.c_double(0)
        self._chk(load().clf_bands_query(self._h, int(what), C.byref(v)), self._h)
        return v.value


def step_static(x, y, coord, depth, a, b, nsteps, dt, eta_max=None, speed2_max=None,
                stream=None, check=True, **params):
    """clf_step_static on torch tensors (argument marshalling only).

    depth: device tensor [ny, nx] in the storage precision; a, b: (h, u, v)
    tuples of device tensors in the storage form (FP64 h; FP32 eta with dry
    nodes at -d).  Returns the index (0 for a, 1 for b) of the buffer that
    holds the final state, and the non-finite flag when `check`."""
    import torch
    L = load()
    x, y = _np64(x), _np64(y)
    ny, nx = depth.shape
    grid = Grid(nx, ny, coord, x.ctypes.data_as(C.POINTER(C.c_double)),
                y.ctypes.data_as(C.POINTER(C.c_double)))
    p = default_params(**params)
    st = stream if stream is not None else torch.cuda.current_stream(depth.device)
    flag = C.c_int(0)
    ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
    rc = L.clf_step_static(C.byref(grid), C.byref(p), float(dt), ptr(depth),
                           *(ptr(t) for t in a), *(ptr(t) for t in b), ptr(eta_max),
                           ptr(speed2_max), int(nsteps), C.c_void_p(st.cuda_stream),
                           C.byref(flag) if check else None)
    if rc != CLF_OK:
        raise ClfError(rc, L.clf_last_error(None).decode())
    return nsteps % 2, (bool(flag.value) if check else None)
