"""Brute-force pin of the FP64 oracle on tiny grids: the whole PonD step
(Sec. IV A-B) is redone here in 40-digit arithmetic (mpmath), with every
transform obtained by inverting the raw-monomial moment matrices of App. B,
and compared with the oracle's double-precision result."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_2302_00310_amd import inputs

mp.mp.dps = 40


class Brute:
    def __init__(self, wl, n_corr):
        self.wl, self.n_corr = wl, n_corr
        self.D = wl.dim
        s6 = mp.sqrt(6)
        c4 = [-mp.sqrt(3 + s6), -mp.sqrt(3 - s6), mp.sqrt(3 - s6), mp.sqrt(3 + s6)]
        w4 = [(3 - s6) / 12, (3 + s6) / 12, (3 + s6) / 12, (3 - s6) / 12]
        c3 = [-mp.sqrt(3), mp.mpf(0), mp.sqrt(3)]
        w3 = [mp.mpf(1) / 6, mp.mpf(2) / 3, mp.mpf(1) / 6]
        self.lat = []
        for c, w in ((c4, w4), (c3, w3)):
            q = len(c)
            if self.D == 1:
                self.lat.append(([(c[k], mp.mpf(0)) for k in range(q)], list(w), q))
            else:
                self.lat.append(([(c[k % q], c[k // q]) for k in range(q * q)],
                                 [w[k % q] * w[k // q] for k in range(q * q)], q))
        self.cv = 1 / (mp.mpf(wl.gamma) - 1)

    # --- App. B transform --------------------------------------------------
    def moment_matrix(self, pop, fr):
        cs, _, q = self.lat[pop]
        rt = mp.sqrt(fr[2])
        M = mp.matrix(len(cs), len(cs))
        nb = q if self.D == 2 else 1
        for b in range(nb):
            for a in range(q):
                r = a + q * b
                for k, (cx, cy) in enumerate(cs):
                    vx, vy = rt * cx + fr[0], rt * cy + fr[1]
                    M[r, k] = vx ** a * (vy ** b if self.D == 2 else 1)
        return M

    def G(self, pop, src, dst):
        return mp.inverse(self.moment_matrix(pop, dst)) * self.moment_matrix(pop, src)

    def tf(self, pop, src, dst, vec):
        out = self.G(pop, src, dst) * mp.matrix(vec)
        return [out[k] for k in range(len(vec))]

    # --- model --------------------------------------------------------------
    def eq(self, rho, T):
        return ([rho * w for w in self.lat[0][1]],
                [(self.cv - mp.mpf(self.D) / 2) * T * rho * w for w in self.lat[1][1]])

    def moments(self, f, g, fr):
        cs = self.lat[0][0]
        rt = mp.sqrt(fr[2])
        m0 = sum(f)
        mx = sum((rt * cx + fr[0]) * fi for (cx, cy), fi in zip(cs, f))
        my = sum((rt * cy + fr[1]) * fi for (cx, cy), fi in zip(cs, f)) if self.D == 2 else 0
        e = sum(((rt * cx + fr[0]) ** 2 + ((rt * cy + fr[1]) ** 2 if self.D == 2 else 0)) / 2 * fi
                for (cx, cy), fi in zip(cs, f)) + sum(g)
        ux, uy = mx / m0, my / m0
        return m0, ux, uy, (e - m0 * (ux * ux + uy * uy) / 2) / (self.cv * m0)

    def qe(self, f, g):
        kappa = self.dt / 2 * (1 / self.tau1 - 1 / self.tau2)
        cs, W, _ = self.lat[0]
        cg, Wg, _ = self.lat[1]
        if self.D == 1:
            h = [cx ** 3 - 3 * cx for cx, _ in cs]
            a3 = sum(fi * hi for fi, hi in zip(f, h))
            ag = sum(gi * cx for gi, (cx, _) in zip(g, cg))
            return ([fi + kappa * w * a3 * hi / 6 for fi, w, hi in zip(f, W, h)],
                    [gi + kappa * w * ag * cx for gi, w, (cx, _) in zip(g, Wg, cg)])
        H = [[cx ** 3 - 3 * cx, cx * cx * cy - cy, cx * cy * cy - cx, cy ** 3 - 3 * cy] for cx, cy in cs]
        al = [sum(fi * h[m] for fi, h in zip(f, H)) for m in range(4)]
        mult = [1, 3, 3, 1]
        agx = sum(gi * cx for gi, (cx, _) in zip(g, cg))
        agy = sum(gi * cy for gi, (_, cy) in zip(g, cg))
        fo = [fi + kappa * w * sum(mult[m] * al[m] * h[m] for m in range(4)) / 6
              for fi, w, h in zip(f, W, H)]
        go = [gi + kappa * w * (agx * cx + agy * cy) for gi, w, (cx, cy) in zip(g, Wg, cg)]
        return fo, go

    def init(self, dt):
        wl = self.wl
        self.dt = mp.mpf(dt)
        self.tau1 = mp.mpf(wl.tau) * self.dt
        self.tau2 = self.tau1 / mp.mpf(wl.prandtl)
        self.dx = mp.mpf(wl.dx)
        r, ux, uy, p = wl.fields()
        self.cells = {}
        for y in range(wl.ny):
            for x in range(wl.nx):
                k = x + wl.nx * y
                rho, T = mp.mpf(r[k]), mp.mpf(p[k]) / mp.mpf(r[k])
                fr = [mp.mpf(ux[k]), mp.mpf(uy[k]) if self.D == 2 else mp.mpf(0), T]
                f, g = self.eq(rho, T)
                self.cells[(x, y)] = [f, g, fr]

    def cell(self, x, y):  # periodic ghosts
        return self.cells[(x % self.wl.nx, y % self.wl.ny)]

    def lim(self, a, b):
        den = abs(a) + abs(b)
        return 0 if den == 0 else (a * abs(b) + abs(a) * b) / den

    def face(self, L, R, LL, RR, Lp, Lm, Rp, Rm, axis, fbp):
        lF = [(L[2][k] + R[2][k]) / 2 for k in range(3)]
        sten = [L, R, LL, RR, Lp, Lm, Rp, Rm] if self.D == 2 else [L, R, LL, RR]
        lam = self.dt / self.dx
        for pss in range(self.n_corr + 1):
            bars = []
            for pop in (0, 1):
                P = [self.tf(pop, c[2], lF, fbp[id(c)][pop]) for c in sten]
                cs = self.lat[pop][0]
                rt = mp.sqrt(lF[2])
                out = []
                for i, (cx, cy) in enumerate(cs):
                    v = [rt * cx + lF[0], rt * cy + lF[1]]
                    vn, vt = v[axis], v[1 - axis]
                    def rec(U, Um, Up, Utm, Utp, dn):
                        val = P[U][i] + dn * self.lim(P[U][i] - P[Um][i], P[Up][i] - P[U][i])
                        if self.D == 2:
                            val += -lam * vt / 2 * self.lim(P[U][i] - P[Utm][i], P[Utp][i] - P[U][i])
                        return val
                    rl = rec(0, 2, 1, 5, 4, mp.mpf(1) / 2 - lam * vn / 2) if self.D == 2 else \
                        rec(0, 2, 1, 0, 0, mp.mpf(1) / 2 - lam * vn / 2)
                    rr = rec(1, 0, 3, 7, 6, -mp.mpf(1) / 2 - lam * vn / 2) if self.D == 2 else \
                        rec(1, 0, 3, 0, 0, -mp.mpf(1) / 2 - lam * vn / 2)
                    band = mp.mpf('1e-11') * rt
                    out.append(rl if vn > band else (rr if vn < -band else (rl + rr) / 2))
                bars.append(out)
            rho_b, ub, vb, Tb = self.moments(bars[0], bars[1], lF)
            if pss < self.n_corr:
                lF = [ub, vb, Tb]
        feqc, geqc = self.eq(rho_b, Tb)
        lb = [ub, vb, Tb]
        feq = self.tf(0, lb, lF, feqc)
        geq = self.tf(1, lb, lF, geqc)
        t, dt = self.tau1, self.dt
        phi_f = [(4 * t * a + dt * e) / (4 * t + dt) for a, e in zip(bars[0], feq)]
        phi_g = [(4 * t * a + dt * e) / (4 * t + dt) for a, e in zip(bars[1], geq)]
        return phi_f, phi_g, lF

    def step(self):
        nx, ny, D = self.wl.nx, self.wl.ny, self.D
        for key in self.cells:
            f, g, fr = self.cells[key]
            self.cells[key][0], self.cells[key][1] = self.qe(f, g)
        t, dt = self.tau1, self.dt
        fbp = {}
        for key, c in self.cells.items():
            rho = sum(c[0])
            feq, geq = self.eq(rho, c[2][2])
            fbp[id(c)] = ([((2 * t - dt / 2) * a + 3 * dt / 2 * e) / (2 * t + dt) for a, e in zip(c[0], feq)],
                          [((2 * t - dt / 2) * a + 3 * dt / 2 * e) / (2 * t + dt) for a, e in zip(c[1], geq)])
        C = self.cell
        fx = {}
        for y in range(ny):
            for i in range(nx + 1):
                fx[(i, y)] = self.face(C(i - 1, y), C(i, y), C(i - 2, y), C(i + 1, y), C(i - 1, y + 1),
                                       C(i - 1, y - 1), C(i, y + 1), C(i, y - 1), 0, fbp)
        fy = {}
        if D == 2:
            for j in range(ny + 1):
                for x in range(nx):
                    fy[(x, j)] = self.face(C(x, j - 1), C(x, j), C(x, j - 2), C(x, j + 1), C(x + 1, j - 1),
                                           C(x - 1, j - 1), C(x + 1, j), C(x - 1, j), 1, fbp)
        b = (2 * t - dt) / (2 * t + dt)
        ce = 2 * dt / (2 * t + dt)
        lam = dt / self.dx
        new = {}
        for (x, y), (f, g, fr) in self.cells.items():
            faces = [(fx[(x, y)], 0, -1), (fx[(x + 1, y)], 0, 1)]
            if D == 2:
                faces += [(fy[(x, y)], 1, -1), (fy[(x, y + 1)], 1, 1)]
            rt = mp.sqrt(fr[2])
            flux = [[0] * len(f), [0] * len(g)]
            for (pf, pg, lF), axis, sign in faces:
                for pop, vec in ((0, pf), (1, pg)):
                    tr = self.tf(pop, lF, fr, vec)
                    for i, (cx, cy) in enumerate(self.lat[pop][0]):
                        vn = rt * cx + fr[0] if axis == 0 else rt * cy + fr[1]
                        flux[pop][i] += sign * vn * tr[i]
            feq, geq = self.eq(sum(f), fr[2])
            f2 = [b * a + ce * e - lam * fl for a, e, fl in zip(f, feq, flux[0])]
            g2 = [b * a + ce * e - lam * fl for a, e, fl in zip(g, geq, flux[1])]
            _, ux, uy, T = self.moments(f2, g2, fr)
            nfr = [ux, uy if D == 2 else mp.mpf(0), T]
            f3, g3 = self.qe(self.tf(0, fr, nfr, f2), self.tf(1, fr, nfr, g2))
            new[(x, y)] = [f3, g3, nfr]
        self.cells = new


def _compare(wl, steps, n_corr):
    o = oracle.Oracle(wl, n_corr=n_corr)
    b = Brute(wl, n_corr)
    b.init(o.dt)
    o.step(steps)
    for _ in range(steps):
        b.step()
    f, g, fr = o.get_state()
    worst = 0.0
    for (x, y), (bf, bg, bfr) in b.cells.items():
        for i in range(len(bf)):
            worst = max(worst, abs(f[i, y, x] - float(bf[i])) / abs(float(bf[i]) + 1e-300) if abs(bf[i]) > 1e-3
                        else abs(f[i, y, x] - float(bf[i])))
        for i in range(len(bg)):
            worst = max(worst, abs(g[i, y, x] - float(bg[i])) / max(abs(float(bg[i])), 1e-3))
        for k in range(3):
            worst = max(worst, abs(fr[k, y, x] - float(bfr[k])) / max(1.0, abs(float(bfr[k]))))
    return worst


def test_bruteforce_1d_two_steps_with_qe_and_corrector():
    wl = inputs.riemann_1d(4, (1.0, 0.3, 1.0), (0.4, -0.2, 0.35), tau=0.8)
    wl.rho[0] = [1.0, 0.7, 0.4, 0.55]
    wl.ux[0] = [0.3, -0.1, -0.2, 0.5]
    wl.p[0] = [1.0, 0.6, 0.35, 0.8]
    wl.prandtl = 0.7
    wl.bc = [inputs.BC_PERIODIC] * 4
    assert _compare(wl, 3, n_corr=1) < 1e-13


def test_bruteforce_2d_one_step():
    rng = np.random.Generator(np.random.PCG64(33))
    wl = inputs.uniform_2d(3, 3, 1.0, 0.0, 0.0, 1.0, prandtl=0.7, tau=0.8)
    wl.rho = rng.uniform(0.4, 1.2, (3, 3))
    wl.ux = rng.uniform(-0.5, 0.5, (3, 3))
    wl.uy = rng.uniform(-0.5, 0.5, (3, 3))
    wl.p = rng.uniform(0.3, 1.0, (3, 3))
    assert _compare(wl, 1, n_corr=0) < 1e-13
