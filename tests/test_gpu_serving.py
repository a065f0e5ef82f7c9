"""Serving: continuous batching of independent solves (pond_server_* through the
C interface).  Each result must be the same alone and in the mix; admission
waits for arena memory; an oversize request is rejected at submit; a solve
that goes non-physical fails alone."""
import time

import numpy as np
import pytest

from paper_2302_00310_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pond():
    import torch
    assert torch.cuda.is_available()
    from paper_2302_00310_amd import pond as p
    p.load_library()
    return p


def _mix():
    return [
        (inputs.vortex_2d(48, steps=1, mach=1.5, noise=1e-3, seed=21, prandtl=0.6, tau=0.6, ny=40), 37),
        (inputs.quadrants_2d(64, steps=1, seed=22, prandtl=0.9, tau=0.52), 50),
        (inputs.quadrants_2d(33, steps=1, seed=23, prandtl=0.71, tau=0.7, ny=47), 20),
        (inputs.vortex_2d(96, steps=1, mach=3.0, noise=1e-3, seed=24, prandtl=1.0, tau=0.55), 64),
        (inputs.quadrants_2d(128, steps=1, seed=25, prandtl=0.5, tau=0.51, ny=64), 45),
    ]


def _alone(pond, wl, steps, transform=0):
    s = pond.Solver(wl, precision=pond.POND_MIXED, transform=transform)
    s.step(steps)
    m = s.moments()
    s.close()
    return [a.reshape(-1) for a in m]


def _serve(pond, jobs, arena_bytes, max_active=64, timeout=120.0, transforms=None, lattices=None,
           precisions=None):
    import torch
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    srv = pond.pond_server_create(arena.data_ptr(), arena_bytes, 0, max_active)
    ids = []
    try:
        for k, (wl, steps) in enumerate(jobs):
            cfg = pond.make_config(wl, precision=precisions[k] if precisions else pond.POND_MIXED,
                                   transform=transforms[k] if transforms else 0,
                                   lattice=lattices[k] if lattices else None)
            ids.append(pond.pond_submit(srv, cfg, *wl.fields(), steps, tag=k))
        out = {}
        t_end = time.time() + timeout
        while len(out) < len(ids):
            assert time.time() < t_end, "serving did not finish"
            for k, rid in enumerate(ids):
                if k in out:
                    continue
                wl, _ = jobs[k]
                rc, m, times = pond.pond_poll(srv, rid, wl.nx * wl.ny)
                if rc != pond.POND_PENDING:
                    out[k] = (rc, m, times)
            time.sleep(0.002)
        return out
    finally:
        pond.pond_server_destroy(srv)
        del arena


def test_each_result_is_the_same_alone_and_in_the_mix(pond):
    jobs = _mix()
    got = _serve(pond, jobs, 1 << 30)
    for k, (wl, steps) in enumerate(jobs):
        rc, m, times = got[k]
        assert rc == pond.POND_OK
        assert times["tag"] == k
        assert times["t_submit"] <= times["t_admit"] <= times["t_done"]
        ref = _alone(pond, wl, steps)
        for a, b in zip(m, ref):
            assert np.array_equal(a, b), k


def test_admission_waits_for_memory(pond):
    jobs = [(inputs.quadrants_2d(96, steps=1, seed=30 + k), 30) for k in range(5)]
    one = pond.pond_state_bytes(pond.make_config(jobs[0][0], precision=pond.POND_MIXED))
    # room for two resident solves (plus the batch table)
    got = _serve(pond, jobs, 2 * one + (1 << 20))
    assert all(got[k][0] == pond.POND_OK for k in range(5))
    t = sorted((got[k][2]["t_admit"], got[k][2]["t_done"]) for k in range(5))
    # at any admission time at most two solves are resident
    for ta, _ in t:
        resident = sum(1 for a, d in t if a <= ta < d)
        assert resident <= 2
    assert max(a for a, _ in t) >= min(d for _, d in t)  # someone waited for memory
    for k, (wl, steps) in enumerate(jobs):
        for a, b in zip(got[k][1], _alone(pond, wl, steps)):
            assert np.array_equal(a, b)


def test_oversize_request_is_rejected(pond):
    import torch
    wl = inputs.quadrants_2d(256, steps=1)
    cfg = pond.make_config(wl, precision=pond.POND_MIXED)
    need = pond.pond_state_bytes(cfg)
    arena = torch.empty(need // 2, dtype=torch.uint8, device="cuda")
    srv = pond.pond_server_create(arena.data_ptr(), need // 2, 0, 4)
    try:
        with pytest.raises(pond.PondError) as e:
            pond.pond_submit(srv, cfg, *wl.fields(), 10)
        assert e.value.code == -5
    finally:
        pond.pond_server_destroy(srv)


def test_a_failing_solve_does_not_touch_the_others(pond):
    jobs = _mix()[:3]
    bad = inputs.quadrants_2d(64, steps=1, seed=99)
    bad.cfl = 12.0  # far beyond the scheme's stability limit
    jobs.insert(1, (bad, 200))
    got = _serve(pond, jobs, 1 << 30)
    assert got[1][0] == -4  # POND_ERR_UNSTABLE
    for k in (0, 2, 3):
        wl, steps = jobs[k]
        assert got[k][0] == pond.POND_OK
        for a, b in zip(got[k][1], _alone(pond, wl, steps)):
            assert np.array_equal(a, b)


def test_lagrange_and_grad_solves_share_a_batch(pond):
    """Solves with either transform resident together (one kernel per
    transform over the same batch table); each result equals its solve
    alone."""
    jobs = _mix()[:4]
    transforms = [1, 0, 1, 0]
    got = _serve(pond, jobs, 1 << 30, transforms=transforms)
    for k, (wl, steps) in enumerate(jobs):
        rc, m, _ = got[k]
        assert rc == pond.POND_OK
        for a, b in zip(m, _alone(pond, wl, steps, transforms[k])):
            assert np.array_equal(a, b), k


def test_input_outside_the_methods_range_is_reported(pond):
    """Request 456 of the 512-solve serving stream (128^2 quadrants, Mach cap
    3.4): across the left half of the horizontal interface the two quadrants
    move apart at 2.4 (in units where the thermal speed is ~0.65), so the
    face-frame transforms reach far outside the node range.  The FP64 oracle
    turns the two rows at the interface non-finite on its first step; the
    GPU step reports POND_ERR_UNSTABLE for the same input, alone and as a
    served request."""
    import oracle
    reqs = inputs.serving_requests(512, sizes=(128, 256, 512, 1024, 2048), materialize=False)
    w = reqs[456].workload
    sub = inputs._rng(5 * 1000 + 456)
    n = int(sub.choice(np.array((128, 256, 512, 1024, 2048))))
    mach = float(sub.uniform(0.5, 4.0))
    wl = inputs.quadrants_2d(n, w.steps, seed=w.seed, tau=w.tau, prandtl=w.prandtl, mach_cap=mach)
    o = oracle.Oracle(wl)
    o.step(1)
    bad = ~np.isfinite(o.moments()[0])
    assert set(np.nonzero(bad)[0]) == {63, 64}
    s = pond.Solver(wl, precision=pond.POND_MIXED)
    try:
        s.step(1)
        with pytest.raises(pond.PondError) as e:
            s.moments()
        assert e.value.code == -4
    finally:
        s.close()
    got = _serve(pond, [(wl, 20)], 1 << 28)
    assert got[0][0] == -4


def test_d2q9_and_forced_solves_share_a_batch(pond):
    """D2Q16 (Lagrange and Grad), D2Q9 and body-force solves in one stream:
    each result equals the same solve run alone, bit for bit (the batch
    launches one step kernel per kind; each skips the others' blocks)."""
    vort = inputs.vortex_2d(40, steps=1, mach=1.0, noise=1e-3, seed=31, ny=36)
    quad = inputs.quadrants_2d(48, steps=1, seed=32, ny=40)
    forced = inputs.vortex_2d(44, steps=1, mach=0.8, noise=1e-3, seed=33, ny=38)
    forced.accel = [0.4, -0.2]
    jobs = [(vort, 30), (quad, 25), (forced, 28), (quad, 22), (vort, 26)]
    transforms = [0, 1, 0, 1, 1]
    lattices = [pond.POND_D2Q16, pond.POND_D2Q9, pond.POND_D2Q16, pond.POND_D2Q16, pond.POND_D2Q9]
    got = _serve(pond, jobs, 1 << 28, transforms=transforms, lattices=lattices)
    for k, (wl, steps) in enumerate(jobs):
        rc, m, _ = got[k]
        assert rc == pond.POND_OK, k
        s = pond.Solver(wl, precision=pond.POND_MIXED, transform=transforms[k], lattice=lattices[k])
        s.step(steps)
        alone = [a.reshape(-1) for a in s.moments()]
        s.close()
        for a, b in zip(m, alone):
            assert np.array_equal(a, b), k


def test_walled_solves_share_a_batch(pond):
    """Walled solves (each launches its ghost-layer kernel before every batched
    step), one of them forced, served beside periodic ones: each result equals
    the same solve alone, bit for bit."""
    couette = inputs.thermal_couette_2d(36, nx=20, steps=1)
    channel = inputs.poiseuille_2d(28, nx=24, steps=1)
    vort = inputs.vortex_2d(40, steps=1, mach=1.0, noise=1e-3, seed=34, ny=36)
    jobs = [(couette, 40), (vort, 30), (channel, 35), (couette, 17)]
    transforms = [0, 1, 1, 1]
    got = _serve(pond, jobs, 1 << 28, transforms=transforms)
    for k, (wl, steps) in enumerate(jobs):
        rc, m, _ = got[k]
        assert rc == pond.POND_OK, k
        for a, b in zip(m, _alone(pond, wl, steps, transforms[k])):
            assert np.array_equal(a, b), k


def test_multiscale_solves_share_a_batch(pond):
    """Multiscale solves (each launches its D2Q9/D2Q16 switch before every
    batched step; a uniform one runs all-D2Q9 steps in the D2Q9 kernel) served
    beside D2Q16 and D2Q9 ones: each result equals the same solve alone, bit
    for bit, and the switch is seen to pick both lattices."""
    quad = inputs.quadrants_2d(48, steps=1, seed=35, ny=40)
    # uniform flow: the switch indicator is zero everywhere (all-D2Q9 steps)
    smooth = inputs.vortex_2d(40, steps=1, mach=0.3, noise=0.0, seed=36, ny=36)
    smooth.rho[:], smooth.ux[:], smooth.uy[:], smooth.p[:] = 1.0, 0.3, -0.1, 1.0
    vort = inputs.vortex_2d(44, steps=1, mach=1.5, noise=1e-3, seed=37, ny=38)
    jobs = [(quad, 30), (smooth, 25), (vort, 28), (quad, 21), (vort, 19)]
    ms = pond.POND_D2Q9_D2Q16
    lattices = [ms, ms, pond.POND_D2Q16, pond.POND_D2Q9, ms]
    transforms = [1] * len(jobs)
    got = _serve(pond, jobs, 1 << 28, transforms=transforms, lattices=lattices)
    q16_cells = {}
    for k, (wl, steps) in enumerate(jobs):
        rc, m, _ = got[k]
        assert rc == pond.POND_OK, k
        s = pond.Solver(wl, precision=pond.POND_MIXED, transform=1, lattice=lattices[k])
        s.step(steps)
        alone = [a.reshape(-1) for a in s.moments()]
        if lattices[k] == ms:
            q16_cells[k] = int((s.lattice_map()[0] == 16).sum())
        s.close()
        for a, b in zip(m, alone):
            assert np.array_equal(a, b), k
    assert q16_cells[1] == 0 and q16_cells[0] > 0


def test_d2q25_solves_are_served(pond):
    """D2Q25 solves run their own kernels inside the served chunk graphs, with
    no tiles in the batched step: mixed with D2Q16 solves, and alone in the
    server (no batched step at all).  Each result equals the same solve
    alone, bit for bit.  The quadrants input of seed 38 (40 x 36) lies
    outside the D2Q25 method's range: the FP64 oracle turns it non-finite on
    its first step, and served it fails alone with POND_ERR_UNSTABLE."""
    quad = inputs.quadrants_2d(40, steps=1, seed=3, ny=36)
    bad = inputs.quadrants_2d(40, steps=1, seed=38, ny=36)
    vort = inputs.vortex_2d(36, steps=1, mach=1.0, noise=1e-3, seed=39, ny=44)
    q25, q16 = pond.POND_D2Q25, pond.POND_D2Q16
    for jobs, lattices in (([(quad, 24), (vort, 30), (bad, 10), (vort, 17)], [q25, q16, q25, q25]),
                           ([(vort, 20), (quad, 13)], [q25, q25])):
        transforms = [1] * len(jobs)
        got = _serve(pond, jobs, 1 << 28, transforms=transforms, lattices=lattices)
        for k, (wl, steps) in enumerate(jobs):
            rc, m, _ = got[k]
            if wl is bad:
                assert rc == -4  # POND_ERR_UNSTABLE
                continue
            assert rc == pond.POND_OK, k
            s = pond.Solver(wl, precision=pond.POND_MIXED, transform=1, lattice=lattices[k])
            s.step(steps)
            alone = [a.reshape(-1) for a in s.moments()]
            s.close()
            for a, b in zip(m, alone):
                assert np.array_equal(a, b), k


def test_fp64_and_1d_solves_are_served(pond):
    """FP64 solves (2D D2Q16, D2Q9 and walled, D2Q25) and 1D solves (both
    precisions) run their own step launches inside the served chunk graphs,
    beside mixed 2D solves in the batched step: each result equals the same
    solve alone, bit for bit."""
    FP64, MIXED = pond.POND_FP64, pond.POND_MIXED
    vort = inputs.vortex_2d(36, steps=1, mach=1.0, noise=1e-3, seed=41, ny=40)
    quad = inputs.quadrants_2d(40, steps=1, seed=3, ny=36)
    couette = inputs.thermal_couette_2d(32, nx=16, steps=1)
    sod = inputs.sod_1d(200, steps=1)
    jobs = [(vort, 21), (quad, 18), (sod, 40), (couette, 25), (sod, 33), (vort, 16), (quad, 12)]
    precisions = [FP64, MIXED, MIXED, FP64, FP64, FP64, FP64]
    lattices = [pond.POND_D2Q16, pond.POND_D2Q16, None, pond.POND_D2Q16, None, pond.POND_D2Q9,
                pond.POND_D2Q25]
    transforms = [0, 1, 0, 1, 0, 1, 1]
    got = _serve(pond, jobs, 1 << 28, transforms=transforms, lattices=lattices,
                 precisions=precisions)
    for k, (wl, steps) in enumerate(jobs):
        rc, m, _ = got[k]
        assert rc == pond.POND_OK, k
        s = pond.Solver(wl, precision=precisions[k], transform=transforms[k], lattice=lattices[k])
        s.step(steps)
        alone = [a.reshape(-1) for a in s.moments()]
        s.close()
        for a, b in zip(m, alone):
            assert np.array_equal(a, b), k


def test_zero_step_requests_return_their_initial_state(pond):
    """nsteps = 0 for every solve kind: the result equals the moments of the
    same solve created and never stepped, bit for bit."""
    FP64, MIXED = pond.POND_FP64, pond.POND_MIXED
    vort = inputs.vortex_2d(24, steps=1, mach=1.0, noise=1e-3, seed=42, ny=20)
    sod = inputs.sod_1d(64, steps=1)
    jobs = [(vort, 0), (sod, 0), (vort, 0), (vort, 0), (vort, 5)]
    precisions = [FP64, MIXED, MIXED, MIXED, MIXED]
    lattices = [pond.POND_D2Q16, None, pond.POND_D2Q25, pond.POND_D2Q9_D2Q16, pond.POND_D2Q16]
    transforms = [0, 0, 1, 1, 0]
    got = _serve(pond, jobs, 1 << 26, transforms=transforms, lattices=lattices,
                 precisions=precisions)
    for k, (wl, steps) in enumerate(jobs):
        rc, m, _ = got[k]
        assert rc == pond.POND_OK, k
        s = pond.Solver(wl, precision=precisions[k], transform=transforms[k], lattice=lattices[k])
        s.step(steps)
        alone = [a.reshape(-1) for a in s.moments()]
        s.close()
        for a, b in zip(m, alone):
            assert np.array_equal(a, b), k
