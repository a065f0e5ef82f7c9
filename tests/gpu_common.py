"""Helpers shared by the GPU tests: run the HIP library and the FP64 oracle on
the same seeded workload and compare."""
import math

import numpy as np

import oracle
from paper_2302_00310_amd import inputs


def solver(wl, precision, **kw):
    from paper_2302_00310_amd import pond
    return pond.Solver(wl, precision=precision, **kw)


def rel_err(a, b, floor=1e-300):
    """max |a - b| / max |b| (scale-relative, safe where b ~ 0)."""
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), floor))


def rel_l2(a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def moment_errors(gpu_m, ora_m, l2=False, u_floor=None):
    """Errors on rho, (u_x, u_y) jointly, T.  u_floor: a velocity scale under
    which the velocity error is taken relative to it (a flow that starts at
    rest has |u| far below its thermal speed, the scale of its rounding)."""
    r_g, ux_g, uy_g, T_g = gpu_m
    r_o, ux_o, uy_o, T_o = ora_m
    f = rel_l2 if l2 else rel_err
    u_g = np.stack([ux_g, uy_g])
    u_o = np.stack([ux_o, uy_o])
    eu = f(u_g, u_o)
    if u_floor is not None:
        scale = np.linalg.norm(u_o) if l2 else np.max(np.abs(u_o))
        if l2:
            eu = float(np.linalg.norm(u_g - u_o) / max(scale, u_floor * np.sqrt(u_o.size)))
        else:
            eu = float(np.max(np.abs(u_g - u_o)) / max(scale, u_floor))
    return {"rho": f(r_g, r_o), "u": eu, "T": f(T_g, T_o)}


def window_samples(wl, points, steps, transform=0, n_corr=0, limiter=0, flat=0,
                   ms_threshold=0.05, dep=2):
    """Oracle values of (rho, u_x, u_y, T) at the cells ``points`` after
    ``steps`` steps, each computed on a window that contains the cell's whole
    domain of dependence (``dep`` cells per step: 2 for the FV stencil, 5 with
    the multiscale switch, whose gradient and dilation add 3), started from
    the same seeded initial fields and advanced with the full grid's dt."""
    dt = oracle.cfl_dt(wl, flat=flat)
    R = dep * steps + 3
    out = []
    for (x, y) in points:
        if wl.dim == 1:
            w, (ox, oy) = inputs.window(wl, x - R, 0, 2 * R + 1, 1)
        else:
            w, (ox, oy) = inputs.window(wl, x - R, y - R, 2 * R + 1, 2 * R + 1)
        o = oracle.Oracle(w, transform=transform, n_corr=n_corr, limiter=limiter, dt=dt, flat=flat,
                          ms_threshold=ms_threshold)
        o.step(steps)
        m = o.moments()
        # position of (x, y) inside the window
        if wl.bc[0] == inputs.BC_PERIODIC:
            ix = R
        else:
            ix = x - ox
        if wl.dim == 1:
            iy = 0
        elif wl.bc[2] == inputs.BC_PERIODIC:
            iy = R
        else:
            iy = y - oy
        out.append(tuple(float(a[iy, ix]) for a in m))
    return np.array(out), dt
