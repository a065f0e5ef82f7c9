"""Parity of the GPU step with the FP64 oracle on the D2Q9 and multiscale
D2Q9/D2Q16 f-lattices (Grad's projection; Sec. III C and IV C).

FP64: moments within 1e-12 of the oracle, the per-cell f-lattice maps equal
and the switch indicator within 1e-12 of the oracle's after every checked
step.  Both sides decide a cell's lattice from the same FP64 indicator; a
flip would need the two indicators to straddle the threshold, and they
differ by rounding only (~1e-15 relative).  Mixed precision: moments within
1e-5 relative L2."""
import numpy as np
import pytest

import oracle
from paper_2302_00310_amd import inputs
from paper_2302_00310_amd.inputs import BC_PERIODIC, BC_ZERO_GRADIENT, Workload

from .gpu_common import moment_errors

pytestmark = pytest.mark.gpu

FP64, MIXED = 0, 1
GRAD = 1
D2Q9, MSCALE = 3, 4          # GPU lattice codes
O_D2Q9, O_MSCALE = 1, 2      # oracle f-lattice codes


@pytest.fixture(scope="module")
def pond():
    import torch
    assert torch.cuda.is_available()
    from paper_2302_00310_amd import pond as p
    p.load_library()
    return p


def lax_tube(nx=64, ny=4):
    left, right = (0.445, 0.698, 3.528), (0.5, 0.0, 0.571)
    w1 = inputs.riemann_1d(nx, left, right)
    rep = lambda a: np.repeat(a, ny, axis=0)
    return Workload("lax", 2, nx, ny, rep(w1.rho), rep(w1.ux), np.zeros((ny, nx)), rep(w1.p),
                    dx=1.0 / nx, bc=[BC_ZERO_GRADIENT, BC_ZERO_GRADIENT, BC_PERIODIC, BC_PERIODIC])


CASES = {
    "lax_64x4": lambda: lax_tube(),
    "quadrants_35x33": lambda: inputs.quadrants_2d(35, steps=1, seed=3, ny=33),
    "vortex_48x40": lambda: inputs.vortex_2d(48, steps=1, noise=1e-3, ny=40, mach=1.0),
    "shu_osher_64x20": lambda: inputs.shu_osher_2d(64, 20, steps=1),
}


@pytest.mark.parametrize("name", list(CASES))
def test_multiscale_fp64_matches_oracle(pond, name):
    wl = CASES[name]()
    print("multiscale fp64", name, flush=True)
    s = pond.Solver(wl, precision=FP64, transform=GRAD, lattice=MSCALE, ms_threshold=0.05)
    o = oracle.Oracle(wl, transform=GRAD, flat=O_MSCALE, ms_threshold=0.05)
    assert s.dt == pytest.approx(o.dt, rel=1e-14)
    try:
        seen16 = seen9 = False
        for _ in range(6):
            s.step(4)
            o.step(4)
            e = moment_errors(s.moments(), o.moments())
            assert max(e.values()) <= 1e-12, e
            qg, tg = s.lattice_map()
            qo, to = o.get_lattice()
            assert np.array_equal(qg, qo)
            np.testing.assert_allclose(tg, to, rtol=1e-12, atol=1e-12 * max(1.0, to.max()))
            seen16 |= bool((qg == 16).any())
            seen9 |= bool((qg == 9).any())
        if name != "vortex_48x40":
            assert seen16 and seen9  # both lattices deployed
    finally:
        s.close()


@pytest.mark.parametrize("name", ["vortex_48x40", "quadrants_35x33"])
def test_d2q9_fp64_matches_oracle(pond, name):
    wl = CASES[name]()
    s = pond.Solver(wl, precision=FP64, transform=GRAD, lattice=D2Q9)
    o = oracle.Oracle(wl, transform=GRAD, flat=O_D2Q9)
    assert s.dt == pytest.approx(o.dt, rel=1e-14)
    try:
        s.step(20)
        o.step(20)
        e = moment_errors(s.moments(), o.moments())
        assert max(e.values()) <= 1e-12, e
        assert (s.lattice_map()[0] == 9).all()
    finally:
        s.close()


@pytest.mark.parametrize("name", ["lax_64x4", "quadrants_35x33"])
def test_multiscale_mixed_matches_oracle(pond, name):
    wl = CASES[name]()
    s = pond.Solver(wl, precision=MIXED, transform=GRAD, lattice=MSCALE, ms_threshold=0.05)
    o = oracle.Oracle(wl, transform=GRAD, flat=O_MSCALE, ms_threshold=0.05)
    try:
        s.step(40)
        o.step(40)
        e = moment_errors(s.moments(), o.moments(), l2=True)
        assert max(e.values()) <= 1e-5, e
    finally:
        s.close()


def test_threshold_zero_is_d2q16_everywhere(pond):
    wl = CASES["quadrants_35x33"]()
    a = pond.Solver(wl, precision=FP64, transform=GRAD, lattice=MSCALE, ms_threshold=0.0)
    b = pond.Solver(wl, precision=FP64, transform=GRAD)
    try:
        a.step(10)
        b.step(10)
        assert (a.lattice_map()[0] == 16).all()
        e = moment_errors(a.moments(), b.moments())
        assert max(e.values()) <= 1e-13, e
    finally:
        a.close()
        b.close()


def test_multiscale_checkpoint_resume_bitwise(pond, tmp_path):
    wl = CASES["lax_64x4"]()
    a = pond.Solver(wl, precision=MIXED, transform=GRAD, lattice=MSCALE)
    b = pond.Solver(wl, precision=MIXED, transform=GRAD, lattice=MSCALE, init=False)
    try:
        a.step(7)
        path = str(tmp_path / "ms.ckpt")
        pond.pond_save(a.h, path)
        pond.pond_load(b.h, path)
        a.step(9)
        b.step(9)
        for x, y in zip(a.moments(), b.moments()):
            assert np.array_equal(x, y)
        assert np.array_equal(a.lattice_map()[0], b.lattice_map()[0])
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("precision", [FP64, MIXED])
def test_multiscale_full_size_shu_osher_sampled_cells(pond, precision):
    """The 4096 x 1024 Shu-Osher channel with the multiscale deployment, 6
    steps: sampled cells against the oracle run on a window holding each
    cell's domain of dependence (5 cells per step)."""
    from .gpu_common import rel_err, window_samples
    wl = inputs.shu_osher_2d()
    steps = 6
    rng = np.random.Generator(np.random.PCG64(23))
    pts = [(0, 0), (wl.nx - 1, wl.ny - 1), (wl.nx // 2, wl.ny // 2), (430, 17), (410, 500)]
    pts += [(int(rng.integers(wl.nx)), int(rng.integers(wl.ny))) for _ in range(3)]
    ref, dt = window_samples(wl, pts, steps, transform=GRAD, flat=O_MSCALE, dep=5)
    print("multiscale full size", precision, flush=True)
    s = pond.Solver(wl, precision=precision, transform=GRAD, lattice=MSCALE, ms_threshold=0.05)
    try:
        assert abs(s.dt / dt - 1.0) < 1e-15
        s.step(steps)
        m = s.moments()
        q = s.lattice_map()[0]
        assert (q == 16).any() and (q == 9).any()
    finally:
        s.close()
    got = np.array([[float(a[y, x]) for a in m] for (x, y) in pts])
    if precision == FP64:
        for k in range(4):
            assert rel_err(got[:, k], ref[:, k], floor=1.0 if k in (1, 2) else 1e-300) <= 1e-12, k
    else:
        # the mixed bar as on whole fields: relative L2 of rho, of (u_x, u_y)
        # jointly and of T over the sampled cells (u_y alone is a small
        # perturbation, so its own relative error is no measure of precision)
        e = moment_errors(tuple(got.T), tuple(ref.T), l2=True)
        assert max(e.values()) <= 1e-5, e
