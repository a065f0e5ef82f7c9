"""Long runs against stored oracle results.

tests/golden/<name>.npz holds (rho, u_x, u_y, T) of the FP64 oracle after
the full number of steps on every second row and column, written by
tests/golden/make_golden.py (which calls only the oracle).  The HIP path runs
the same seeded workload for the same steps through the C interface, in FP64
and in mixed precision, and is compared on those cells: FP64 within 1e-12
relative to the field's magnitude, mixed within 1e-5 relative L2 on rho, u and
T."""
import os

import numpy as np
import pytest

from paper_2302_00310_amd import inputs

from .gpu_common import moment_errors

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

CASES = {
    "vortex_256_1000": lambda: inputs.vortex_2d(256, steps=1000),
    "quadrants_256_500": lambda: inputs.quadrants_2d(256, steps=500),
    "shu_osher_512x128_500": lambda: inputs.shu_osher_2d(512, 128, steps=500),
}
TOL = {0: 1e-12, 1: 1e-5}  # FP64 (max, relative), mixed (L2, relative)


@pytest.fixture(scope="module")
def pond():
    import torch
    assert torch.cuda.is_available()
    from paper_2302_00310_amd import pond as p
    p.load_library()
    return p


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", [0, 1])
def test_long_run_matches_stored_oracle(pond, name, precision):
    path = os.path.join(HERE, name + ".npz")
    ref = np.load(path)
    wl = CASES[name]()
    stride = int(ref["stride"])
    print(f"golden {name} precision={precision} steps={int(ref['steps'])}", flush=True)
    s = pond.Solver(wl, precision=precision)
    try:
        assert s.dt == pytest.approx(float(ref["dt"]), rel=1e-14)
        s.step(int(ref["steps"]))
        got = [np.ascontiguousarray(a[::stride, ::stride]) for a in s.moments()]
    finally:
        s.close()
    want = [ref["rho"], ref["ux"], ref["uy"], ref["T"]]
    err = moment_errors(got, want, l2=precision == 1)
    print(name, precision, err, flush=True)
    assert max(err.values()) <= TOL[precision], err
