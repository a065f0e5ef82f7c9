"""ctypes wrapper of oracle/libpondref.so (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

TF_LAGRANGE, TF_GRAD = 0, 1
LIM_VANLEER, LIM_MINMOD = 0, 1
F_D2Q16, F_D2Q9, F_MULTISCALE, F_D2Q25 = 0, 1, 2, 3
MS_THRESHOLD = 0.05  # default switch threshold of the multiscale deployment


class OracleConfig(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("transform", C.c_int),
                ("gamma", C.c_double), ("tau", C.c_double), ("prandtl", C.c_double),
                ("cfl", C.c_double), ("dx", C.c_double), ("bc", C.c_int * 4),
                ("inflow", (C.c_double * 4) * 4), ("limiter", C.c_int), ("n_corr", C.c_int),
                ("flat", C.c_int), ("ms_threshold", C.c_double),
                ("wall", (C.c_double * 3) * 4), ("accel", C.c_double * 2)]


_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def load_library():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.path.join(_HERE, "libpondref.so")
    if not os.path.exists(path):
        from .build import build
        build()
    lib = C.CDLL(path)
    lib.pondref_last_error.restype = C.c_char_p
    lib.pondref_create.argtypes = [C.POINTER(OracleConfig), C.POINTER(C.c_void_p)]
    lib.pondref_destroy.argtypes = [C.c_void_p]
    lib.pondref_destroy.restype = None
    lib.pondref_init_fields.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
    lib.pondref_cfl_dt.argtypes = [C.POINTER(OracleConfig), _dp, _dp, _dp, _dp]
    lib.pondref_cfl_dt.restype = C.c_double
    lib.pondref_set_dt.argtypes = [C.c_void_p, C.c_double]
    lib.pondref_get_dt.argtypes = [C.c_void_p]
    lib.pondref_get_dt.restype = C.c_double
    lib.pondref_step.argtypes = [C.c_void_p, C.c_int]
    lib.pondref_moments.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
    lib.pondref_totals.argtypes = [C.c_void_p, _dp]
    lib.pondref_get_state.argtypes = [C.c_void_p, _dp, _dp, _dp]
    lib.pondref_set_state.argtypes = [C.c_void_p, _dp, _dp, _dp]
    lib.pondref_get_faces.argtypes = [C.c_void_p, _dp, _dp, _dp, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.pondref_set_threads.argtypes = [C.c_int]
    lib.pondref_lattice.argtypes = [C.c_int, _dp, _dp]
    lib.pondref_transform_matrix.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp]
    lib.pondref_transform_matrix_full.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp]
    lib.pondref_qe_half_step.argtypes = [C.c_int, C.c_double, _dp, _dp]
    lib.pondref_ms_matrix.argtypes = [C.c_int, _dp, C.c_int, _dp, _dp]
    lib.pondref_get_lattice.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    lib.pondref_wall_ghost.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, _dp, _dp, _dp]
    _LIB = lib
    return lib


def _check(rc):
    if rc < 0:
        raise RuntimeError("pondref: " + load_library().pondref_last_error().decode())
    return rc


def make_config(wl, transform=TF_LAGRANGE, limiter=LIM_VANLEER, n_corr=0, flat=F_D2Q16,
                ms_threshold=MS_THRESHOLD) -> OracleConfig:
    c = OracleConfig()
    c.dim, c.nx, c.ny = wl.dim, wl.nx, wl.ny
    c.transform = transform
    c.gamma, c.tau, c.prandtl, c.cfl, c.dx = wl.gamma, wl.tau, wl.prandtl, wl.cfl, wl.dx
    for k in range(4):
        c.bc[k] = int(wl.bc[k])
        for m in range(4):
            c.inflow[k][m] = float(wl.inflow[k][m])
    c.limiter, c.n_corr = limiter, n_corr
    c.flat, c.ms_threshold = flat, ms_threshold
    wall = getattr(wl, "wall", None)
    if wall is not None:
        for k in range(4):
            for m in range(3):
                c.wall[k][m] = float(wall[k][m])
    accel = getattr(wl, "accel", None)
    if accel is not None:
        c.accel[0], c.accel[1] = float(accel[0]), float(accel[1])
    return c


def set_threads(n: int) -> int:
    return load_library().pondref_set_threads(int(n))


def get_threads() -> int:
    return load_library().pondref_get_threads()


_Q1 = {0: 4, 1: 3, 2: 5}   # nodes of lattice_get's rules: D1Q4, D1Q3, D1Q5


def lattice(which: int):
    c = np.zeros(5)
    w = np.zeros(5)
    q = _check(load_library().pondref_lattice(which, c, w))
    return c[:q].copy(), w[:q].copy()


def transform_matrix(dim, which, src, dst, transform=TF_LAGRANGE):
    q = _Q1[which]
    Q = q ** dim
    G = np.zeros(Q * Q)
    _check(load_library().pondref_transform_matrix(dim, which, transform,
                                                   np.ascontiguousarray(src, float), np.ascontiguousarray(dst, float), G))
    return G.reshape(Q, Q)


def transform_matrix_full(dim, which, src, dst):
    q = _Q1[which]
    Q = q ** dim
    G = np.zeros(Q * Q)
    _check(load_library().pondref_transform_matrix_full(dim, which, np.ascontiguousarray(src, float),
                                                        np.ascontiguousarray(dst, float), G))
    return G.reshape(Q, Q)


def ms_matrix(q1s, src, q1t, dst):
    """Multiscale frame transformation between 2D f-lattices (q1 = 4: D2Q16,
    3: D2Q9); rows = target populations."""
    G = np.zeros(q1t * q1t * q1s * q1s)
    _check(load_library().pondref_ms_matrix(q1s, np.ascontiguousarray(src, float), q1t,
                                            np.ascontiguousarray(dst, float), G))
    return G.reshape(q1t * q1t, q1s * q1s)


def cfl_dt(wl, flat=F_D2Q16) -> float:
    """The CFL step of ``wl``'s initial fields on the f-lattice ``flat`` (the
    D2Q9 f-lattices need Grad's projection, so the config names it)."""
    cfg = make_config(wl, TF_GRAD if flat != F_D2Q16 else TF_LAGRANGE, flat=flat)
    r, a, b, p = wl.fields()
    dt = load_library().pondref_cfl_dt(C.byref(cfg), r, a, b, p)
    if not dt > 0.0:
        raise RuntimeError("pondref: " + load_library().pondref_last_error().decode())
    return dt


class Oracle:
    """One oracle solve; ``wl`` is an ``inputs.Workload``."""

    def __init__(self, wl, transform=TF_LAGRANGE, limiter=LIM_VANLEER, n_corr=0, dt=None,
                 init=True, flat=F_D2Q16, ms_threshold=MS_THRESHOLD):
        self.lib = load_library()
        self.wl = wl
        self.cfg = make_config(wl, transform, limiter, n_corr, flat, ms_threshold)
        h = C.c_void_p()
        _check(self.lib.pondref_create(C.byref(self.cfg), C.byref(h)))
        self.h = h
        self.dim, self.nx, self.ny = wl.dim, wl.nx, wl.ny
        self.Qf, self.Qg = (4, 3) if wl.dim == 1 else (25 if flat == F_D2Q25 else 16, 9)
        if dt is not None:
            _check(self.lib.pondref_set_dt(self.h, float(dt)))
        if init:
            _check(self.lib.pondref_init_fields(self.h, *wl.fields()))

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.pondref_destroy(self.h)
            self.h = None

    @property
    def dt(self) -> float:
        return self.lib.pondref_get_dt(self.h)

    def step(self, n: int = 1):
        _check(self.lib.pondref_step(self.h, int(n)))

    def moments(self):
        n = self.nx * self.ny
        out = [np.zeros(n) for _ in range(4)]
        _check(self.lib.pondref_moments(self.h, *out))
        return tuple(a.reshape(self.ny, self.nx) for a in out)

    def totals(self):
        out = np.zeros(4)
        _check(self.lib.pondref_totals(self.h, out))
        return out

    def get_state(self):
        n = self.nx * self.ny
        f = np.zeros(self.Qf * n)
        g = np.zeros(self.Qg * n)
        fr = np.zeros(3 * n)
        _check(self.lib.pondref_get_state(self.h, f, g, fr))
        return (f.reshape(self.Qf, self.ny, self.nx), g.reshape(self.Qg, self.ny, self.nx),
                fr.reshape(3, self.ny, self.nx))

    def set_state(self, f, g, fr):
        _check(self.lib.pondref_set_state(self.h, np.ascontiguousarray(f, float).reshape(-1),
                                          np.ascontiguousarray(g, float).reshape(-1),
                                          np.ascontiguousarray(fr, float).reshape(-1)))

    def get_lattice(self):
        """Per cell: f population count (16 or 9) and the last switch indicator."""
        n = self.nx * self.ny
        q = np.zeros(n, dtype=np.int32)
        th = np.zeros(n)
        _check(self.lib.pondref_get_lattice(self.h, q.ctypes.data, th.ctypes.data))
        return q.reshape(self.ny, self.nx), th.reshape(self.ny, self.nx)

    def wall_ghost(self, side, layer, t):
        """(f~, g~, frame) of ghost layer ``layer`` of wall ``side`` at
        coordinate ``t`` along the wall, from the current state."""
        f, g, fr = np.zeros(16), np.zeros(9), np.zeros(3)
        _check(self.lib.pondref_wall_ghost(self.h, side, layer, t, f, g, fr))
        return f, g, fr

    def get_faces(self):
        nx, ny = self.nx, self.ny
        nfx = (nx + 1) * ny
        fx = np.zeros(nfx * self.Qf)
        gx = np.zeros(nfx * self.Qg)
        lx = np.zeros(nfx * 3)
        if self.dim == 2:
            nfy = nx * (ny + 1)
            fy = np.zeros(nfy * self.Qf)
            gy = np.zeros(nfy * self.Qg)
            ly = np.zeros(nfy * 3)
            _check(self.lib.pondref_get_faces(self.h, fx, gx, lx, fy.ctypes.data, gy.ctypes.data,
                                              ly.ctypes.data))
            return (fx.reshape(nfx, self.Qf), gx.reshape(nfx, self.Qg), lx.reshape(nfx, 3),
                    fy.reshape(nfy, self.Qf), gy.reshape(nfy, self.Qg), ly.reshape(nfy, 3))
        _check(self.lib.pondref_get_faces(self.h, fx, gx, lx, None, None, None))
        return fx.reshape(nfx, self.Qf), gx.reshape(nfx, self.Qg), lx.reshape(nfx, 3)


def qe_half_step(dim, kappa, f, g):
    f = np.array(f, dtype=np.float64)
    g = np.array(g, dtype=np.float64)
    _check(load_library().pondref_qe_half_step(dim, float(kappa), f, g))
    return f, g
