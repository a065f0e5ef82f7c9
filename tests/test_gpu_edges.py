"""Edge cases of the GPU step against the FP64 oracle: zero steps leave the
state untouched, and the smallest grids the library accepts (4 cells per
axis) match the oracle on every f-lattice, with walls and with a body force
(a 4-cell axis is narrower than the 16 x 15 tile and the two-cell halo)."""
import numpy as np
import pytest

import oracle
from paper_2302_00310_amd import inputs
from paper_2302_00310_amd.inputs import BC_PERIODIC, BC_WALL, BC_ZERO_GRADIENT, Workload

from .gpu_common import moment_errors

pytestmark = pytest.mark.gpu

FP64, MIXED = 0, 1


@pytest.fixture(scope="module")
def pond():
    import torch
    assert torch.cuda.is_available()
    from paper_2302_00310_amd import pond as p
    p.load_library()
    return p


def tiny(nx=4, ny=4, seed=9):
    rng = np.random.default_rng(seed)
    f = lambda lo, hi: rng.uniform(lo, hi, (ny, nx))
    return Workload("tiny", 2, nx, ny, f(0.5, 1.5), f(-0.5, 0.5), f(-0.5, 0.5), f(0.5, 1.5),
                    prandtl=0.7, dx=1.0 / nx, bc=[BC_ZERO_GRADIENT, BC_ZERO_GRADIENT, BC_PERIODIC, BC_PERIODIC])


def test_zero_steps_leave_the_state_untouched(pond):
    wl = inputs.quadrants_2d(35, steps=1, seed=3, ny=33)
    s = pond.Solver(wl, precision=MIXED)
    try:
        m0 = s.moments()
        s.step(0)
        m1 = s.moments()
        assert all(np.array_equal(a, b) for a, b in zip(m0, m1))
    finally:
        s.close()


KINDS = {
    "d2q16_lagrange": dict(gpu={}, ora={}),
    "d2q16_grad": dict(gpu={"transform": 1}, ora={"transform": 1}),
    "d2q9": dict(gpu={"transform": 1, "lattice": 3}, ora={"transform": 1, "flat": 1}),
    "multiscale": dict(gpu={"transform": 1, "lattice": 4}, ora={"transform": 1, "flat": 2}),
    "d2q25": dict(gpu={"transform": 1, "lattice": 5}, ora={"transform": 1, "flat": 3}),
}


@pytest.mark.parametrize("kind", list(KINDS))
def test_smallest_grid_matches_oracle(pond, kind):
    wl = tiny()
    k = KINDS[kind]
    print("edge 4x4", kind, flush=True)
    s = pond.Solver(wl, precision=FP64, **k["gpu"])
    o = oracle.Oracle(wl, **k["ora"])
    try:
        s.step(6)
        o.step(6)
        e = moment_errors(s.moments(), o.moments())
        assert max(e.values()) <= 1e-12, e
    finally:
        s.close()


def test_smallest_grid_with_walls_and_force(pond):
    wl = tiny()
    rng = np.random.default_rng(10)
    # temperatures near the walls' (a mirrored ghost temperature 2 T_w - T_B
    # must stay positive)
    wl.p = wl.rho * rng.uniform(0.95, 1.05, wl.rho.shape)
    wl.bc = [BC_PERIODIC, BC_PERIODIC, BC_WALL, BC_WALL]
    wl.wall = [[0, 0, 1.0], [0, 0, 1.0], [0, 0, 1.0], [0.2, 0, 1.1]]
    wl.accel = [0.3, -0.1]
    s = pond.Solver(wl, precision=FP64)
    o = oracle.Oracle(wl)
    try:
        s.step(6)
        o.step(6)
        e = moment_errors(s.moments(), o.moments(), u_floor=1.0)
        assert max(e.values()) <= 1e-12, e
    finally:
        s.close()


def test_smallest_1d_grid_matches_oracle(pond):
    wl = inputs.sod_1d(4, steps=1)
    s = pond.Solver(wl, precision=FP64)
    o = oracle.Oracle(wl)
    try:
        s.step(8)
        o.step(8)
        e = moment_errors(s.moments(), o.moments(), u_floor=1.0)
        assert max(e.values()) <= 1e-12, e
    finally:
        s.close()
