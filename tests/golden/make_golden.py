"""Write the stored expected values of the long parity runs.

Runs only the FP64 oracle (oracle/) on the seeded workloads below and
stores (rho, u_x, u_y, T) after the stated number of steps, on every second
row and column of the grid, in tests/golden/<name>.npz.  Usage:

    python tests/golden/make_golden.py [name ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2302_00310_amd import inputs  # noqa: E402

CASES = {
    # isentropic vortex advected at Mach 2, 256^2 periodic, Pr 0.71, 1000 steps
    "vortex_256_1000": (lambda: inputs.vortex_2d(256, steps=1000), 1000),
    # four-quadrant state (seed 3) on 256^2, zero gradient, 500 steps
    "quadrants_256_500": (lambda: inputs.quadrants_2d(256, steps=500), 500),
    # Mach-3 shock into the sinusoidal field, 512 x 128 channel, 500 steps
    "shu_osher_512x128_500": (lambda: inputs.shu_osher_2d(512, 128, steps=500), 500),
}
STRIDE = 2


def make(name):
    build, steps = CASES[name]
    wl = build()
    o = oracle.Oracle(wl)
    t0 = time.time()
    o.step(steps)
    m = o.moments()
    sub = [np.ascontiguousarray(a[::STRIDE, ::STRIDE]) for a in m]
    np.savez_compressed(os.path.join(HERE, name + ".npz"), rho=sub[0], ux=sub[1], uy=sub[2],
                        T=sub[3], steps=steps, stride=STRIDE, dt=o.dt)
    print(f"{name}: {steps} steps in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    for n in names:
        make(n)
