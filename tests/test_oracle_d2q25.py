"""Pins of the oracle's D2Q25 f-lattice with the fourth-order Grad
projection (Sec. III B, full invariant moment system; Table I; Sec. V shock
structure).

The D1Q5 rule is the five-point Gauss--Hermite rule; the fourth-order
projection keeps every moment of total order <= 4; the projected comoving
equilibrium has the Maxwell--Boltzmann moments up to fourth order in any
frame (closed forms), so the fourth-order moment R that D2Q16 gets wrong
away from the comoving frame (eq. DeviationR) is exact here; the update
conserves mass, momentum and energy (App. C: K >= 3), keeps a uniform flow
at any Mach number, and converges to the exact Riemann solution on the
Lax tube."""
import math
import os
import sys

import numpy as np
import pytest
from numpy.polynomial import hermite_e as He

import oracle
from paper_2302_00310_amd import inputs
from paper_2302_00310_amd.inputs import BC_PERIODIC, BC_ZERO_GRADIENT, Workload

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import exact_riemann  # noqa: E402

GRAD = oracle.pondref.TF_GRAD
Q25 = oracle.F_D2Q25
RNG = np.random.default_rng(25)


def test_d1q5_is_the_five_point_gauss_hermite_rule():
    c, w = oracle.lattice(2)
    x, wx = He.hermegauss(5)
    np.testing.assert_allclose(c, x, atol=1e-15)
    np.testing.assert_allclose(w, wx / math.sqrt(2 * math.pi), atol=1e-16)


def tensor5():
    c, w = oracle.lattice(2)
    cx = np.array([c[i % 5] for i in range(25)])
    cy = np.array([c[i // 5] for i in range(25)])
    W = np.array([w[i % 5] * w[i // 5] for i in range(25)])
    return cx, cy, W


def raw(f, fr, order):
    cx, cy, _ = tensor5()
    vx, vy = math.sqrt(fr[2]) * cx + fr[0], math.sqrt(fr[2]) * cy + fr[1]
    return {(a, b): np.sum(f * vx ** a * vy ** b) for a in range(order + 1) for b in range(order + 1 - a)}


def frame():
    return np.array([RNG.uniform(-1.5, 1.5), RNG.uniform(-1.5, 1.5), RNG.uniform(0.3, 2.5)])


def test_fourth_order_projection_keeps_moments_to_order_four():
    for _ in range(6):
        src, dst = frame(), frame()
        f = RNG.uniform(0.0, 1.0, 25)
        G = oracle.transform_matrix(2, 2, src, dst, transform=GRAD)
        ms, md = raw(f, src, 4), raw(G @ f, dst, 4)
        for k in ms:
            assert md[k] == pytest.approx(ms[k], rel=1e-11, abs=1e-11), k


def maxwell_moment(a, b, u, T):
    """E[v_x^a v_y^b] of the unit-density Maxwellian (u, T): product of 1D
    Gaussian moments sum_k C(a,k) u^(a-k) T^(k/2) (k-1)!! for even k."""
    def m1(n, m):
        return sum(math.comb(n, k) * m ** (n - k) * T ** (k / 2) * (math.prod(range(k - 1, 0, -2)) if k else 1)
                   for k in range(0, n + 1, 2))
    return m1(a, u[0]) * m1(b, u[1])


def test_projected_equilibrium_has_maxwell_moments_to_fourth_order():
    """The comoving equilibrium rho W in frame lambda, projected to another
    frame: on D2Q25 every moment of total order <= 4 is the Maxwellian's;
    on D2Q16 the fourth-order ones are not (the R deviation)."""
    _, _, W25 = tensor5()
    c4, w4 = oracle.lattice(0)
    W16 = np.array([w4[i % 4] * w4[i // 4] for i in range(16)])
    for _ in range(4):
        lam, bar = frame(), frame()
        f25 = oracle.transform_matrix(2, 2, lam, bar, transform=GRAD) @ W25
        m25 = raw(f25, bar, 4)
        for (a, b), v in m25.items():
            assert v == pytest.approx(maxwell_moment(a, b, lam[:2], lam[2]), rel=1e-11, abs=1e-11)
        f16 = oracle.transform_matrix(2, 0, lam, bar, transform=GRAD) @ W16
        cx4 = np.array([c4[i % 4] for i in range(16)])
        vx = math.sqrt(bar[2]) * cx4 + bar[0]
        dev = abs(np.sum(f16 * vx ** 4) - maxwell_moment(4, 0, lam[:2], lam[2]))
        assert dev > 1e-4


def box25(n=12, mach=0.0, seed=0):
    x = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(x, x)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
    u0 = mach * math.sqrt(1.4)
    ux = u0 + 0.3 * np.cos(2 * np.pi * Y)
    uy = 0.2 * np.sin(2 * np.pi * X)
    T = 1.0 + 0.1 * np.cos(2 * np.pi * (X + Y))
    return Workload("box25", 2, n, n, rho, ux, uy, rho * T, prandtl=0.7, tau=0.6, dx=1.0 / n,
                    bc=[BC_PERIODIC] * 4)


def test_d2q25_conserves_mass_momentum_energy():
    o = oracle.Oracle(box25(), transform=GRAD, flat=Q25)
    t0 = o.totals()
    o.step(15)
    np.testing.assert_allclose(o.totals(), t0, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("mach", [0.0, 3.0])
def test_d2q25_uniform_flow_stays_uniform(mach):
    u = mach * math.sqrt(1.4) / math.sqrt(2.0)
    o = oracle.Oracle(inputs.uniform_2d(6, 6, 1.0, u, -u, 1.0), transform=GRAD, flat=Q25)
    o.step(10)
    r, ux, uy, T = o.moments()
    for a, v in ((r, 1.0), (ux, u), (uy, -u), (T, 1.0)):
        np.testing.assert_allclose(a, v, rtol=1e-13, atol=1e-13)


def test_d2q25_lax_tube_converges_to_the_exact_solution():
    left, right = (0.445, 0.698, 3.528), (0.5, 0.0, 0.571)
    err = {}
    for nx in (40, 80):
        w1 = inputs.riemann_1d(nx, left, right)
        wl = Workload("lax", 2, nx, 1, w1.rho, w1.ux, np.zeros((1, nx)), w1.p, dx=1.0 / nx,
                      bc=[BC_ZERO_GRADIENT, BC_ZERO_GRADIENT, BC_PERIODIC, BC_PERIODIC])
        o = oracle.Oracle(wl, transform=GRAD, flat=Q25)
        n = int(round(0.08 / o.dt))
        o.step(n)
        x = (np.arange(nx) + 0.5) / nx
        exact = exact_riemann.solution(left, right, 1.4, x, 0.5, n * o.dt)[0]
        err[nx] = np.mean(np.abs(o.moments()[0][0] - exact))
    assert err[40] < 0.06, err
    assert err[80] < 0.75 * err[40], err


def test_d2q25_config_rules():
    wl = box25()
    with pytest.raises(RuntimeError):
        oracle.Oracle(wl, transform=0, flat=Q25)
