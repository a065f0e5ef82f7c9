"""Exact solution of the 1D Riemann problem of the Euler equations for an
ideal gas (textbook construction: two-shock/rarefaction star-state pressure
by Newton iteration, then self-similar sampling).  Test helper only."""
import math

import numpy as np


def _fk(p, rho, pk, ck, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        f = (p - pk) * math.sqrt(A / (p + B))
        df = math.sqrt(A / (B + p)) * (1.0 - 0.5 * (p - pk) / (B + p))
    else:  # rarefaction
        f = 2.0 * ck / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho * ck) * (p / pk) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(left, right, g):
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    p = max(1e-12, 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr))
    for _ in range(100):
        fl, dfl = _fk(p, rl, pl, cl, g)
        fr, dfr = _fk(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(1e-14, p - dp)
        if abs(pn - p) < 1e-14 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, cl, g)
    fr, _ = _fk(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(left, right, g, xi):
    """(rho, u, p) at x/t = xi."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us = star_state(left, right, g)
    if xi <= us:  # left of contact
        if ps > pl:  # left shock
            sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
            if xi <= sl:
                return rl, ul, pl
            r = rl * ((ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1))
            return r, us, ps
        shl = ul - cl
        cs = cl * (ps / pl) ** ((g - 1) / (2 * g))
        stl = us - cs
        if xi <= shl:
            return rl, ul, pl
        if xi >= stl:
            return rl * (ps / pl) ** (1 / g), us, ps
        c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - xi))
        u = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + xi)
        r = rl * (c / cl) ** (2 / (g - 1))
        return r, u, pl * (c / cl) ** (2 * g / (g - 1))
    if ps > pr:  # right shock
        sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
        if xi >= sr:
            return rr, ur, pr
        r = rr * ((ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1))
        return r, us, ps
    shr = ur + cr
    cs = cr * (ps / pr) ** ((g - 1) / (2 * g))
    str_ = us + cs
    if xi >= shr:
        return rr, ur, pr
    if xi <= str_:
        return rr * (ps / pr) ** (1 / g), us, ps
    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - xi))
    u = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + xi)
    r = rr * (c / cr) ** (2 / (g - 1))
    return r, u, pr * (c / cr) ** (2 * g / (g - 1))


def solution(left, right, g, x, x0, t):
    out = np.array([sample(left, right, g, (xx - x0) / t) for xx in x])
    return out[:, 0], out[:, 1], out[:, 2]
