"""Thin ctypes binding of libpond.so (include/pond.h).

Functions carry the C names and only marshal arguments; every step of the
PonD time step runs in the library's HIP kernels.  PyTorch provides the
device arena (a uint8 CUDA tensor) and the HIP stream.  The library must be
built (``paper_2302_00310_amd/build.py``); there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpond.so")

POND_OK, POND_PENDING = 0, 1
ERRORS = {-1: "POND_ERR_INVALID", -2: "POND_ERR_NOMEM", -3: "POND_ERR_DEVICE",
          -4: "POND_ERR_UNSTABLE", -5: "POND_ERR_REJECTED", -6: "POND_ERR_UNSUPPORTED"}
POND_D1Q4, POND_D2Q16, POND_D2Q9, POND_D2Q9_D2Q16, POND_D2Q25 = 1, 2, 3, 4, 5
POND_FP64, POND_MIXED = 0, 1
POND_TF_LAGRANGE, POND_TF_GRAD = 0, 1
POND_BC_PERIODIC, POND_BC_ZERO_GRADIENT, POND_BC_INFLOW, POND_BC_WALL = 0, 1, 2, 3
POND_LIM_VANLEER, POND_LIM_MINMOD = 0, 1


class PondError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class pond_config(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("lattice", C.c_int),
                ("transform", C.c_int), ("precision", C.c_int), ("gamma", C.c_double),
                ("tau", C.c_double), ("prandtl", C.c_double), ("cfl", C.c_double),
                ("dx", C.c_double), ("bc", C.c_int * 4), ("inflow", (C.c_double * 4) * 4),
                ("limiter", C.c_int), ("n_corr", C.c_int), ("ms_threshold", C.c_double),
                ("wall", (C.c_double * 3) * 4), ("accel", C.c_double * 2)]


_dbl = C.POINTER(C.c_double)


class pond_request(C.Structure):
    _fields_ = [("cfg", pond_config), ("rho", _dbl), ("ux", _dbl), ("uy", _dbl), ("p", _dbl),
                ("nsteps", C.c_int), ("tag", C.c_uint64)]


class pond_result(C.Structure):
    _fields_ = [("status", C.c_int), ("rho", _dbl), ("ux", _dbl), ("uy", _dbl), ("T", _dbl),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("tag", C.c_uint64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpond.so.  torch is imported first so that the library binds to
    the same HIP runtime as torch's tensors and streams."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (HIP runtime shared with torch)
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: run paper_2302_00310_amd/build.py")
    lib = C.CDLL(path)
    vp, sz, i, d = C.c_void_p, C.c_size_t, C.c_int, C.c_double
    dp = C.POINTER(C.c_double)
    sig = {
        "pond_last_error": ([C.c_char_p, sz], i),
        "pond_state_bytes": ([C.POINTER(pond_config)], sz),
        "pond_create": ([C.POINTER(pond_config), vp, sz, vp, C.POINTER(vp)], i),
        "pond_init_fields": ([vp, dp, dp, dp, dp], i),
        "pond_step": ([vp, i], i),
        "pond_moments": ([vp, dp, dp, dp, dp], i),
        "pond_totals": ([vp, dp], i),
        "pond_totals_fixed": ([vp, C.POINTER(C.c_int64), C.POINTER(C.c_int)], i),
        "pond_export_state": ([vp, dp, dp, dp], i),
        "pond_get_time": ([vp, dp, C.POINTER(C.c_int64)], i),
        "pond_save": ([vp, C.c_char_p], i),
        "pond_load": ([vp, C.c_char_p], i),
        "pond_destroy": ([vp], i),
        "pond_lattice_constants": ([dp], i),
        "pond_server_create": ([vp, sz, vp, i, C.POINTER(vp)], i),
        "pond_submit": ([vp, C.POINTER(pond_request), C.POINTER(C.c_uint64)], i),
        "pond_poll": ([vp, C.c_uint64, C.POINTER(pond_result)], i),
        "pond_server_stats": ([vp, C.POINTER(C.c_double)], i),
        "pond_lattice_map": ([vp, C.POINTER(C.c_int), C.POINTER(C.c_double)], i),
        "pond_server_destroy": ([vp], i),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def exported_symbols():
    """Names declared in include/pond.h that the binding expects."""
    return ["pond_last_error", "pond_state_bytes", "pond_create", "pond_init_fields", "pond_step",
            "pond_moments", "pond_totals", "pond_totals_fixed", "pond_export_state",
            "pond_get_time", "pond_save", "pond_load", "pond_destroy", "pond_lattice_constants",
            "pond_lattice_map",
            "pond_server_create", "pond_submit", "pond_poll", "pond_server_stats",
            "pond_server_destroy"]


def last_error() -> str:
    buf = C.create_string_buffer(512)
    load_library().pond_last_error(buf, 512)
    return buf.value.decode()


def check(rc: int) -> int:
    if rc < 0:
        raise PondError(rc, last_error())
    return rc


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dbl)


def _host(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(-1)


# ---- the C functions, same names ------------------------------------------
def pond_state_bytes(cfg: pond_config) -> int:
    return load_library().pond_state_bytes(C.byref(cfg))


def pond_create(cfg: pond_config, dev_arena: int, arena_bytes: int, hip_stream: int):
    h = C.c_void_p()
    check(load_library().pond_create(C.byref(cfg), C.c_void_p(dev_arena), arena_bytes,
                                     C.c_void_p(hip_stream), C.byref(h)))
    return h


def pond_init_fields(h, rho, ux, uy, p):
    rho, ux, uy, p = (_host(a) for a in (rho, ux, uy, p))
    return check(load_library().pond_init_fields(h, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(p)))


def pond_step(h, nsteps: int):
    return check(load_library().pond_step(h, int(nsteps)))


def pond_moments(h, n: int):
    out = [np.empty(n) for _ in range(4)]
    rc = load_library().pond_moments(h, *[_ptr(a) for a in out])
    return rc, out


def pond_totals(h):
    out = np.zeros(4)
    return check(load_library().pond_totals(h, _ptr(out))), out


def pond_totals_fixed(h):
    out = (C.c_int64 * 8)()
    bits = C.c_int()
    rc = check(load_library().pond_totals_fixed(h, out, C.byref(bits)))
    return rc, [int(out[2 * q]) * 2 ** 64 + (int(out[2 * q + 1]) & (2 ** 64 - 1)) for q in range(4)], bits.value


def pond_export_state(h, n: int, qf: int, qg: int):
    f = np.empty(qf * n)
    g = np.empty(qg * n)
    fr = np.empty(3 * n)
    rc = load_library().pond_export_state(h, _ptr(f), _ptr(g), _ptr(fr))
    return rc, f, g, fr


def pond_lattice_map(h, nx: int, ny: int):
    q = np.zeros(nx * ny, dtype=np.int32)
    th = np.zeros(nx * ny)
    check(load_library().pond_lattice_map(h, q.ctypes.data_as(C.POINTER(C.c_int)),
                                          th.ctypes.data_as(C.POINTER(C.c_double))))
    return q.reshape(ny, nx), th.reshape(ny, nx)


def pond_get_time(h):
    dt = C.c_double()
    ns = C.c_int64()
    check(load_library().pond_get_time(h, C.byref(dt), C.byref(ns)))
    return dt.value, ns.value


def pond_save(h, path: str):
    return check(load_library().pond_save(h, path.encode()))


def pond_load(h, path: str):
    return check(load_library().pond_load(h, path.encode()))


def pond_destroy(h):
    return check(load_library().pond_destroy(h))


def pond_lattice_constants():
    out = np.zeros(14)
    check(load_library().pond_lattice_constants(_ptr(out)))
    return out


# ---- convenience -----------------------------------------------------------
def make_config(wl, precision=POND_FP64, transform=POND_TF_LAGRANGE, limiter=POND_LIM_VANLEER,
                n_corr=0, lattice=None, ms_threshold=0.05) -> pond_config:
    """pond_config of an ``inputs.Workload``; lattice defaults to D1Q4 / D2Q16."""
    c = pond_config()
    c.dim, c.nx, c.ny = wl.dim, wl.nx, wl.ny
    c.lattice = lattice if lattice is not None else (POND_D1Q4 if wl.dim == 1 else POND_D2Q16)
    c.ms_threshold = ms_threshold
    c.transform, c.precision = transform, precision
    c.gamma, c.tau, c.prandtl, c.cfl, c.dx = wl.gamma, wl.tau, wl.prandtl, wl.cfl, wl.dx
    for k in range(4):
        c.bc[k] = int(wl.bc[k])
        for m in range(4):
            c.inflow[k][m] = float(wl.inflow[k][m])
    wall = getattr(wl, "wall", None)
    if wall is not None:
        for k in range(4):
            for m in range(3):
                c.wall[k][m] = float(wall[k][m])
    accel = getattr(wl, "accel", None)
    if accel is not None:
        c.accel[0], c.accel[1] = float(accel[0]), float(accel[1])
    c.limiter, c.n_corr = limiter, n_corr
    return c


class Solver:
    """One solve on the current torch device and stream."""

    def __init__(self, wl, precision=POND_FP64, n_corr=0, limiter=POND_LIM_VANLEER,
                 transform=POND_TF_LAGRANGE, stream=None, init=True, lattice=None,
                 ms_threshold=0.05):
        import torch
        self.wl = wl
        self.cfg = make_config(wl, precision, transform, limiter, n_corr, lattice, ms_threshold)
        self.bytes = pond_state_bytes(self.cfg)
        if self.bytes == 0:
            load_library()
            check(load_library().pond_create(C.byref(self.cfg), None, 0, None, C.byref(C.c_void_p())))
        self.arena = torch.empty(self.bytes, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.h = pond_create(self.cfg, self.arena.data_ptr(), self.bytes, self.stream.cuda_stream)
        self.n = wl.nx * wl.ny
        self.qf, self.qg = (4, 3) if wl.dim == 1 else (25 if self.cfg.lattice == POND_D2Q25 else 16, 9)
        if init:
            pond_init_fields(self.h, *wl.fields())

    def step(self, n: int = 1):
        pond_step(self.h, n)

    def moments(self, check_status=True):
        rc, out = pond_moments(self.h, self.n)
        if check_status:
            check(rc)
        return tuple(a.reshape(self.wl.ny, self.wl.nx) for a in out)

    def lattice_map(self):
        """Per cell: f population count (16 or 9) and the last switch indicator."""
        return pond_lattice_map(self.h, self.wl.nx, self.wl.ny)

    def export_state(self):
        rc, f, g, fr = pond_export_state(self.h, self.n, self.qf, self.qg)
        check(rc)
        sh = (self.wl.ny, self.wl.nx)
        return f.reshape(self.qf, *sh), g.reshape(self.qg, *sh), fr.reshape(3, *sh)

    def totals(self):
        return pond_totals(self.h)[1]

    def totals_fixed(self):
        return pond_totals_fixed(self.h)[1]

    @property
    def dt(self):
        return pond_get_time(self.h)[0]

    def close(self):
        if getattr(self, "h", None) is not None:
            pond_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- serving ----------------------------------------------------------------
def pond_server_create(dev_arena: int, arena_bytes: int, hip_stream: int, max_active: int):
    h = C.c_void_p()
    check(load_library().pond_server_create(C.c_void_p(dev_arena), arena_bytes,
                                            C.c_void_p(hip_stream), int(max_active), C.byref(h)))
    return h


def pond_submit(srv, cfg: pond_config, rho, ux, uy, p, nsteps: int, tag: int = 0) -> int:
    req = pond_request()
    req.cfg = cfg
    arrs = [_host(a) for a in (rho, ux, uy, p)]
    req.rho, req.ux, req.uy, req.p = (_ptr(a) for a in arrs)
    req.nsteps = int(nsteps)
    req.tag = int(tag)
    rid = C.c_uint64()
    check(load_library().pond_submit(srv, C.byref(req), C.byref(rid)))
    return rid.value


def pond_poll(srv, rid: int, n: int):
    """(status, (rho, ux, uy, T) or None, times dict or None); status 1 = pending."""
    res = pond_result()
    out = [np.empty(n) for _ in range(4)]
    res.rho, res.ux, res.uy, res.T = (_ptr(a) for a in out)
    rc = load_library().pond_poll(srv, C.c_uint64(rid), C.byref(res))
    if rc == POND_PENDING:
        return rc, None, None
    if rc < 0 and res.t_submit == 0.0 and res.t_done == 0.0:
        raise PondError(rc, last_error())
    times = {"t_submit": res.t_submit, "t_admit": res.t_admit, "t_done": res.t_done, "tag": res.tag}
    return rc, out, times


def pond_server_stats(srv) -> dict:
    out = (C.c_double * 9)()
    check(load_library().pond_server_stats(srv, out))
    keys = ("elapsed_s", "cell_updates", "chunks", "set_changes", "admit_s", "retire_s",
            "table_s", "capture_s", "gpu_s")
    return dict(zip(keys, list(out)))


def pond_server_destroy(srv):
    return check(load_library().pond_server_destroy(srv))
