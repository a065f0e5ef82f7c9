"""Parity of the GPU step with the FP64 oracle under a body force (App. D:
Strang half steps of d f / dt = F around the kinetic update, explicit Euler
with the re-gauge to the new comoving frame), on a periodic box, beside
zero-gradient sides, and in the force-driven channel between walls, with
both frame transformations.  FP64 within 1e-12, mixed within 1e-5 relative
L2; the full 2048^2 box on sampled cells."""
import numpy as np
import pytest

import oracle
from paper_2302_00310_amd import inputs
from paper_2302_00310_amd.inputs import Workload

from .gpu_common import moment_errors, window_samples

pytestmark = pytest.mark.gpu

FP64, MIXED = 0, 1


@pytest.fixture(scope="module")
def pond():
    import torch
    assert torch.cuda.is_available()
    from paper_2302_00310_amd import pond as p
    p.load_library()
    return p


def forced(wl, accel):
    return Workload(wl.name + "_forced", 2, wl.nx, wl.ny, wl.rho, wl.ux, wl.uy, wl.p, gamma=wl.gamma,
                    tau=wl.tau, prandtl=wl.prandtl, dx=wl.dx if wl.dx > 0 else 1.0 / wl.nx,
                    bc=list(wl.bc), inflow=[list(r) for r in wl.inflow],
                    wall=[list(r) for r in wl.wall], accel=list(accel), steps=wl.steps)


def channel(ny=33, nx=20):
    wl = inputs.poiseuille_2d(ny=ny, nx=nx, u_max=0.05, reynolds=2.0)
    wl.tau = 0.025 / oracle.cfl_dt(wl)
    wl.prandtl = 0.7
    return wl


CASES = {
    "vortex_box_37x33": lambda: forced(inputs.vortex_2d(37, steps=1, noise=1e-3, ny=33, mach=1.0),
                                       (0.5, -0.3)),
    "quadrants_35x33": lambda: forced(inputs.quadrants_2d(35, steps=1, seed=3, ny=33), (0.2, 0.4)),
    "channel_20x33": channel,
}


@pytest.mark.parametrize("transform", [0, 1])
@pytest.mark.parametrize("name", list(CASES))
def test_force_fp64_matches_oracle(pond, name, transform):
    wl = CASES[name]()
    print("force fp64", name, transform, flush=True)
    s = pond.Solver(wl, precision=FP64, transform=transform)
    o = oracle.Oracle(wl, transform=transform)
    assert s.dt == pytest.approx(o.dt, rel=1e-14)
    try:
        for _ in range(3):
            s.step(7)
            o.step(7)
            # velocities relative to max(|u|, 1): the channel starts at rest,
            # its thermal speed (T = 1) sets the scale of rounding
            e = moment_errors(s.moments(), o.moments(), u_floor=1.0)
            assert max(e.values()) <= 1e-12, e
    finally:
        s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_force_mixed_matches_oracle(pond, name):
    wl = CASES[name]()
    s = pond.Solver(wl, precision=MIXED)
    o = oracle.Oracle(wl)
    try:
        s.step(40)
        o.step(40)
        e = moment_errors(s.moments(), o.moments(), l2=True, u_floor=1.0)
        assert max(e.values()) <= 1e-5, e
    finally:
        s.close()


def test_uniform_gas_accelerates_exactly(pond):
    wl = forced(inputs.uniform_2d(20, 17, 1.0, 0.1, -0.2, 1.0), (0.3, 0.7))
    s = pond.Solver(wl, precision=FP64)
    try:
        s.step(30)
        r, ux, uy, T = s.moments()
        dt = s.dt
    finally:
        s.close()
    t = 30 * dt
    np.testing.assert_allclose(ux, 0.1 + 0.3 * t, atol=1e-13)
    np.testing.assert_allclose(uy, -0.2 + 0.7 * t, atol=1e-13)
    cool = 60 * dt ** 2 * (0.3 ** 2 + 0.7 ** 2) / (8 / 0.4)   # 60 half steps, 8 C_v = 20
    np.testing.assert_allclose(T, 1.0 - cool, rtol=1e-13)


def test_force_full_size_sampled_cells(pond):
    v = inputs.vortex_2d(2048, steps=4, noise=1e-3, mach=1.0)
    wl = forced(v, (0.5, -0.3))
    steps = 4
    n = wl.nx
    pts = [(0, 0), (n - 1, n - 1), (n // 2, n // 2), (300, 1700), (1999, 5)]
    for precision in (FP64, MIXED):
        print("force full size", precision, flush=True)
        ref, dt = window_samples(wl, pts, steps)
        s = pond.Solver(wl, precision=precision)
        try:
            assert abs(s.dt / dt - 1.0) < 1e-15
            s.step(steps)
            m = s.moments()
        finally:
            s.close()
        got = np.array([[float(a[y, x]) for a in m] for (x, y) in pts])
        e = moment_errors(tuple(got.T), tuple(ref.T), l2=(precision == MIXED))
        assert max(e.values()) <= (1e-12 if precision == FP64 else 1e-5), (precision, e)


def test_force_driven_channel_reaches_the_parabolic_profile_on_the_gpu(pond):
    """16 cells across, Re 2, 5,600 steps (0.75 viscous times).  The FP64 GPU
    step is within 1e-12 of the oracle after 1,000 steps; both FP64 and
    mixed meet the parabolic profile within 2.5% at the end (the oracle's
    pin).  The scheme itself amplifies rounding-size differences in this
    flow (the oracle started from densities perturbed by 1e-15 differs from
    itself by ~1e-11 after 3,000 steps and ~1e-8 after 5,600), so element
    parity is checked where that growth is still below the bar."""
    u_max, nu = 0.05, 0.025
    wl = inputs.poiseuille_2d(ny=16, u_max=u_max, reynolds=u_max / nu)
    dt = oracle.cfl_dt(wl)
    wl.tau = nu / dt
    steps = int(0.75 / (nu * dt))
    o = oracle.Oracle(wl)
    o.step(1000)
    y = (np.arange(16) + 0.5) / 16
    for precision in (FP64, MIXED):
        s = pond.Solver(wl, precision=precision)
        try:
            s.step(1000)
            if precision == FP64:
                e = moment_errors(s.moments(), o.moments(), u_floor=1.0)
                assert max(e.values()) <= 1e-12, e
            s.step(steps - 1000)
            m = s.moments()
        finally:
            s.close()
        assert np.abs(m[1][:, 0] - 4 * u_max * y * (1 - y)).max() / u_max < 0.025


def test_forced_channel_checkpoint_resume_bitwise(pond, tmp_path):
    """Walls and a body force: a solve saved after 7 steps and loaded into a
    fresh state continues bit for bit."""
    wl = CASES["channel_20x33"]()
    a = pond.Solver(wl, precision=MIXED)
    b = pond.Solver(wl, precision=MIXED, init=False)
    try:
        a.step(7)
        path = str(tmp_path / "ch.ckpt")
        pond.pond_save(a.h, path)
        pond.pond_load(b.h, path)
        a.step(9)
        b.step(9)
        for x, y in zip(a.moments(), b.moments()):
            assert np.array_equal(x, y)
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("transform", [0, 1])
def test_force_with_a_corrector_pass(pond, transform):
    wl = CASES["vortex_box_37x33"]()
    s = pond.Solver(wl, precision=FP64, transform=transform, n_corr=1)
    o = oracle.Oracle(wl, transform=transform, n_corr=1)
    try:
        s.step(10)
        o.step(10)
        e = moment_errors(s.moments(), o.moments(), u_floor=1.0)
        assert max(e.values()) <= 1e-12, e
    finally:
        s.close()
