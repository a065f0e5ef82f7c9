"""Benchmark of the PonD time step on one MI355X.

Workload: the four-quadrant 2D Riemann stand-in, 2048 x 2048 cells,
D2Q16 f + D2Q9 g, zero-gradient boundaries, Pr = 0.71, tau = 0.55, seeded
states (seed 3).  The headline value is the mixed-precision step (FP32
populations, FP64 gauge and conservative fluxes); the FP64 step is timed on
the same grid for the mixed/FP64 speed-up.  Inputs are resident in HBM before
the timed region.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# gfx950: 256 CUs x 4 SIMD x 16 lanes x 2 flops (FMA) x 2.4 GHz.  Packed FP32
# is not used (the kernels are compiled without packed FP32 instructions), so FP32
# and FP64 vector ops share this peak.
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

# Algorithmic bytes per 2D cell-update: the persistent state read once and
# written once -- 25 non-equilibrium populations plus the 4 x 64-bit
# conserved-moment ledger.
BYTES_PER_CELL = {"mixed": 2 * (25 * 4 + 4 * 8), "fp64": 2 * (25 * 8 + 4 * 8)}

# Measured HBM bytes per launch of step_batch_kernel<2,float> on this workload
# (2048^2): rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE in separate runs, scaled
# by 2.0 and 1.0, the factors that make the same counters read 1 GiB for a
# 1 GiB device copy (the counter summary kept with the profiles).
# The figures belong to the kernel sources with the digest below; for any
# other source the traffic is reported as null.
KERNEL_SOURCES = ("paper_2302_00310_amd/csrc/pond_kernels.hip",
                  "paper_2302_00310_amd/csrc/pond_internal.h")
MEASURED_TRAFFIC = {
    "sha256": "99dcd79c640ca4cf7b5615da5def6e4ebca0329a8b198f629b94455f783bdf35",
    "n": 2048,
    "fetch_bytes": 1.64760e+09,
    "write_bytes": 7.89201e+08,
}


def kernel_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(n: int):
    """HBM bytes per launch from the recorded counters, or None when the
    kernel sources or the grid differ from the ones they were taken on."""
    m = MEASURED_TRAFFIC
    if n != m["n"] or kernel_digest() != m["sha256"]:
        return None
    return m["fetch_bytes"] + m["write_bytes"]


def flops_per_cell_2d(n_corr: int = 0) -> int:
    """Floating-point operations of one 2D cell-update as the kernel's
    algorithm specifies them (FMA = 2).  Per face (two per cell), for each
    of the 8 stencil cells: the Lagrange factors of the f transform
    (2 x 4 points x 15) plus its 2 x 64 FMA application, and the same for g
    (2 x 3 points x 10, 2 x 27 FMA); reconstruction (25 populations x 24);
    FP64 face moments (16 x 10 + 9); face equilibrium (f: 2 x 4 points x 23,
    g: 2 x 3 points x 16, 25 x 4 for the products and the inversion);
    conserved fluxes (16 x 12 + 9 x 3).  Per cell: four face-to-cell
    transforms and one re-gauge (5 x (376 + 168)), flux products and update
    (25 x 8), two quasi-equilibrium half steps (2 x 300), phi-bar-plus and
    frames (60)."""
    f_tf = 2 * 4 * 15 + 2 * 64 * 2
    g_tf = 2 * 3 * 10 + 2 * 27 * 2
    stencil = 8 * (f_tf + g_tf)
    per_pass = stencil + 25 * 24 + (16 * 10 + 9)
    face = (1 + n_corr) * per_pass + (2 * 4 * 23 + 2 * 3 * 16 + 25 * 4) + (16 * 12 + 9 * 3)
    cell = 5 * (f_tf + g_tf) + 25 * 8 + 2 * 300 + 60
    return 2 * face + cell


def flops_per_cell_d2q25() -> int:
    """Floating-point operations of one D2Q25 cell-update as its kernels
    specify them (FMA = 2, n_corr = 0).  Grad's map of order 4 on D2Q25:
    Hermite values at the 2 x 5 shifted nodes (2 x 5 x 5), the moment stage
    (125 + 75 FMA) and the expansion (75 + 100 FMA); of order 2 on D2Q9:
    (2 x 3 x 3) + (27 + 18 + 18 + 18 FMA).  Per face (two per cell): 8
    stencil projections, reconstruction (34 x 30), FP64 face moments
    (25 x 10 + 9), face equilibrium (34 products and one projection),
    inversion and fluxes (34 x 2 + 25 x 10 + 9 x 2).  Per cell: the cell pass
    (QE half step 25 x 10 + 9 x 4, phi-bar-plus 34 x 2, frame 30), four
    face-to-cell projections with their flux products (34 x 3), the update
    (34 x 4), the re-gauge projection and the second QE half step."""
    f_map = 2 * 5 * 5 + 2 * (125 + 75 + 75 + 100)
    g_map = 2 * 3 * 3 + 2 * (27 + 18 + 18 + 18)
    proj = f_map + g_map
    face = 8 * proj + 34 * 30 + (25 * 10 + 9) + (34 + proj) + (34 * 2 + 25 * 10 + 9 * 2)
    qe = 25 * 10 + 9 * 4
    cell = (qe + 34 * 2 + 30) + 4 * (proj + 34 * 3) + 34 * 4 + proj + qe + 30
    return 2 * face + cell


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--n", type=int, default=2048, help="grid side")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-fp64", action="store_true")
    p.add_argument("--no-multiscale", action="store_true",
                   help="skip the multiscale D2Q9/D2Q16 leg")
    p.add_argument("--no-walls", action="store_true", help="skip the wall-boundary leg")
    p.add_argument("--no-force", action="store_true", help="skip the body-force leg")
    p.add_argument("--no-d2q25", action="store_true", help="skip the D2Q25 leg")
    p.add_argument("--cpu-seconds", type=float, default=20.0)
    p.add_argument("--serving-requests", type=int, default=64,
                   help="requests of the serving leg (0 skips it)")
    p.add_argument("--serving-sizes", type=str, default="128,256,512",
                   help="grid sides drawn uniformly by the serving leg")
    p.add_argument("--serving-arena-gb", type=float, default=16.0)
    p.add_argument("--serving-max-active", type=int, default=64)
    p.add_argument("--copy-mb", type=int, default=0,
                   help="after timing, copy this many MiB device-to-device (counter calibration)")
    return p.parse_args()


def time_path(wl, precision, steps, warmup, **solver_kw):
    import torch
    from paper_2302_00310_amd import pond
    s = pond.Solver(wl, precision=precision, **solver_kw)
    stream = torch.cuda.current_stream()
    s.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = e0.elapsed_time(e1) / steps
    rc, _ = pond.pond_moments(s.h, s.n)  # surfaces any non-physical state
    pond.check(rc)
    if solver_kw.get("lattice") == pond.POND_D2Q9_D2Q16:
        time_path.d2q16_fraction = float((s.lattice_map()[0] == 16).mean())
    s.close()
    return wall, kern_ms


def multiscale_leg(steps, warmup):
    """The multiscale D2Q9/D2Q16 deployment (Grad's projection, switch
    threshold 0.05) against D2Q16 and D2Q9 everywhere with the same
    transform (mixed precision), on the Shu-Osher channel 4096 x 1024 and on
    the advected vortex 2048^2.  The multiscale step includes its two switch
    kernels."""
    from paper_2302_00310_amd import inputs, pond
    res = {}
    for key, wl, desc in (
            ("shu_osher_4096x1024", inputs.shu_osher_2d(4096, 1024, steps=1),
             "Shu-Osher channel 4096x1024, inflow Mach 3 shock into a sinusoidal density field "
             "with a random phase per row (seed 4)"),
            ("vortex_2048", inputs.vortex_2d(2048, steps=1),
             "isentropic vortex advected at Mach 2, 2048^2 periodic (seed 2)")):
        cells = wl.nx * wl.ny
        out = {"workload": desc + "; mixed precision, Grad's projection"}
        for name, kw in (("d2q16", {}), ("d2q9", {"lattice": pond.POND_D2Q9}),
                         ("multiscale", {"lattice": pond.POND_D2Q9_D2Q16, "ms_threshold": 0.05})):
            wall, kern = time_path(wl, pond.POND_MIXED, steps, warmup,
                                   transform=pond.POND_TF_GRAD, **kw)
            out[name] = {"value": cells * steps / wall, "unit": "cell-updates/s",
                         "ms_per_step": kern}
        out["multiscale"]["d2q16_cell_fraction"] = time_path.d2q16_fraction
        out["multiscale_over_d2q16"] = out["multiscale"]["value"] / out["d2q16"]["value"]
        res[key] = out
    return res


def cpu_baseline(wl_full, seconds):
    """The FP64 oracle as it stands, on the host cores, on a 256 x 256 window
    of the same workload (domain centre), advanced with the full grid's dt."""
    import oracle
    from paper_2302_00310_amd import inputs
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    threads = oracle.set_threads(cores)
    dt = oracle.cfl_dt(wl_full)
    n = 256
    w, _ = inputs.window(wl_full, wl_full.nx // 2 - n // 2, wl_full.ny // 2 - n // 2, n, n)
    o = oracle.Oracle(w, dt=dt)
    t0 = time.perf_counter()
    o.step(1)
    one = time.perf_counter() - t0
    steps = max(1, int(seconds / max(one, 1e-3)))
    t0 = time.perf_counter()
    o.step(steps)
    el = time.perf_counter() - t0
    return {"value": n * n * steps / el, "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n}x{n} window at the centre of the 2048^2 quadrant workload, "
                      f"{steps} FP64 steps in {el:.1f} s"}


def serving_leg(n_req, sizes, arena_gb, max_active):
    """Poisson stream of independent mixed-precision solves (rate 50/s, seed 5)
    through the serving loop: submit at each arrival time, poll until done.
    Latency = t_done - t_submit on the server's clock."""
    import numpy as np
    import torch
    from paper_2302_00310_amd import inputs, pond
    reqs = inputs.serving_requests(n_req, sizes=sizes)
    arena_bytes = int(arena_gb * (1 << 30))
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    srv = pond.pond_server_create(arena.data_ptr(), arena_bytes, 0, max_active)
    ids, results = [], {}
    cells_steps = 0
    t0 = time.perf_counter()
    k = 0
    try:
        while len(results) < len(reqs):
            now = time.perf_counter() - t0
            while k < len(reqs) and reqs[k].arrival <= now:
                wl = reqs[k].workload
                cfg = pond.make_config(wl, precision=pond.POND_MIXED)
                ids.append(pond.pond_submit(srv, cfg, *wl.fields(), wl.steps, tag=k))
                cells_steps += wl.nx * wl.ny * wl.steps
                k += 1
            for j, rid in enumerate(ids):
                if j in results:
                    continue
                wl = reqs[j].workload
                rc, _, times = pond.pond_poll(srv, rid, wl.nx * wl.ny)
                if rc != pond.POND_PENDING:
                    results[j] = (rc, times)
                    print(f"serving: {len(results)}/{len(reqs)} done", file=sys.stderr, flush=True)
            time.sleep(0.001)
        makespan = time.perf_counter() - t0
        stats = pond.pond_server_stats(srv)
    finally:
        pond.pond_server_destroy(srv)
    lat = np.array([r[1]["t_done"] - r[1]["t_submit"] for r in results.values()])
    queue = np.array([r[1]["t_admit"] - r[1]["t_submit"] for r in results.values()])
    serv = np.array([r[1]["t_done"] - r[1]["t_admit"] for r in results.values()])
    failed = [[j, int(r[0]), reqs[j].workload.nx, reqs[j].workload.name]
              for j, r in sorted(results.items()) if r[0] != 0]
    return {"requests": len(reqs), "ok": int(sum(1 for r in results.values() if r[0] == 0)),
            "failed": failed,
            "sizes": list(sizes), "rate_per_s": 50.0, "arena_gb": arena_gb,
            "max_active": max_active, "policy": "FCFS with memory admission",
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "queue_p50_s": float(np.percentile(queue, 50)), "queue_p99_s": float(np.percentile(queue, 99)),
            "service_p50_s": float(np.percentile(serv, 50)), "service_p99_s": float(np.percentile(serv, 99)),
            "throughput_cell_updates_per_s": cells_steps / makespan, "makespan_s": makespan,
            "server": stats}


def walls_leg(n, steps, warmup):
    """Wall boundaries (mirrored Chapman-Enskog ghost cells, one ghost kernel
    per step before the step kernel), mixed precision, Lagrange maps: the
    thermal Couette channel n^2 (walls along y, periodic x) and a closed box
    n^2 (walls on all sides, moving lid, the advected-vortex field), each
    against the same fields on a periodic grid."""
    from paper_2302_00310_amd import inputs, pond
    from paper_2302_00310_amd.inputs import BC_PERIODIC, BC_WALL, Workload
    cells = n * n
    cou = inputs.thermal_couette_2d(ny=n, nx=n, prandtl=0.71, eckert=4.0)
    v = inputs.vortex_2d(n, steps=1, mach=0.5)
    box = Workload("walled_box", 2, n, n, v.rho, v.ux, v.uy, v.p, tau=v.tau, prandtl=v.prandtl,
                   dx=1.0 / n, bc=[BC_WALL] * 4,
                   wall=[[0, 0, 1.0], [0, 0, 1.0], [0, 0, 1.0], [0.3, 0, 1.1]])
    res = {}
    for key, wl, desc in (
            ("thermal_couette", cou, f"thermal Couette channel {n}x{n}, Ma 0.5, Ec 4, Pr 0.71"),
            ("walled_box", box, f"closed box {n}x{n}, lid 0.3, isentropic vortex at Mach 0.5")):
        per = Workload(wl.name + "_periodic", 2, n, n, wl.rho, wl.ux, wl.uy, wl.p, tau=wl.tau,
                       prandtl=wl.prandtl, dx=wl.dx, bc=[BC_PERIODIC] * 4)
        out = {"workload": desc + "; mixed precision"}
        for name, w in (("walls", wl), ("periodic", per)):
            wall, kern = time_path(w, pond.POND_MIXED, steps, warmup)
            out[name] = {"value": cells * steps / wall, "unit": "cell-updates/s",
                         "ms_per_step": kern}
        out["walls_over_periodic"] = out["walls"]["value"] / out["periodic"]["value"]
        res[key] = out
    return res


def force_leg(n, steps, warmup):
    """Body force (two Strang half steps per step, each an Euler update and a
    re-gauge, fused into the step kernel), mixed precision, Lagrange maps:
    the advected vortex n^2 with and without a constant acceleration, and the
    force-driven channel n^2 between walls (Re 2)."""
    from paper_2302_00310_amd import inputs, pond
    from paper_2302_00310_amd.inputs import Workload
    cells = n * n
    v = inputs.vortex_2d(n, steps=1)
    acc = Workload("vortex_forced", 2, n, n, v.rho, v.ux, v.uy, v.p, tau=v.tau, prandtl=v.prandtl,
                   dx=v.dx, bc=list(v.bc), accel=[0.5, -0.3])
    ch = inputs.poiseuille_2d(ny=n, nx=n, u_max=0.05, reynolds=2.0)
    ch.tau = 0.55
    out = {"workload": f"isentropic vortex {n}^2 at Mach 2 (seed 2) with a = (0.5, -0.3); "
                       f"force-driven channel {n}x{n} between walls; mixed precision"}
    for name, w in (("vortex_forced", acc), ("vortex_unforced", v), ("channel", ch)):
        wall, kern = time_path(w, pond.POND_MIXED, steps, warmup)
        out[name] = {"value": cells * steps / wall, "unit": "cell-updates/s", "ms_per_step": kern}
    out["forced_over_unforced"] = out["vortex_forced"]["value"] / out["vortex_unforced"]["value"]
    return out


def d2q25_leg(n, steps, warmup):
    """The D2Q25 f-lattice with the fourth-order Grad projection (three plain
    kernels per step with the face data in HBM) against the fused D2Q16 step
    with Grad's projection, on the four-quadrant workload n^2, mixed and
    FP64."""
    from paper_2302_00310_amd import inputs, pond
    wl = inputs.quadrants_2d(n, steps=steps)
    cells = n * n
    out = {"workload": f"four-quadrant 2D Riemann stand-in {n}x{n} (seed 3), Grad's projection"}
    for name, prec, lat in (("d2q25_mixed", pond.POND_MIXED, pond.POND_D2Q25),
                            ("d2q25_fp64", pond.POND_FP64, pond.POND_D2Q25),
                            ("d2q16_mixed", pond.POND_MIXED, pond.POND_D2Q16)):
        wall, kern = time_path(wl, prec, steps, warmup, transform=pond.POND_TF_GRAD, lattice=lat)
        out[name] = {"value": cells * steps / wall, "unit": "cell-updates/s", "ms_per_step": kern}
    out["d2q25_over_d2q16_mixed"] = out["d2q25_mixed"]["value"] / out["d2q16_mixed"]["value"]
    flops = flops_per_cell_d2q25()
    for name in ("d2q25_mixed", "d2q25_fp64"):
        tf = flops * cells / (out[name]["ms_per_step"] * 1e-3) / 1e12
        out[name]["alu_roofline"] = {"bound": "alu", "achieved": tf, "peak": VALU_PEAK_TFLOPS,
                                     "unit": "TFLOP/s", "frac": tf / VALU_PEAK_TFLOPS,
                                     "flops_per_cell": flops}
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2302_00310_amd import inputs, pond
    pond.load_library()
    wl = inputs.quadrants_2d(a.n, steps=a.steps)
    cells = wl.nx * wl.ny

    wall_m, kern_m = time_path(wl, pond.POND_MIXED, a.steps, a.warmup)
    value = cells * a.steps / wall_m
    out = {
        "metric": "cell-updates/s mixed vs FP64 step (% HBM roofline); p50/p99 solve latency",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1e3 * wall_m / a.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"four-quadrant 2D Riemann stand-in, {a.n}x{a.n}, D2Q16+D2Q9, "
                               "zero-gradient, Pr=0.71, tau=0.55, seed 3, mixed precision "
                               "(FP32 populations, FP64 gauge/fluxes), n_corr=0",
                   "cells": cells},
    }
    flops = flops_per_cell_2d(0)
    achieved_tf = flops * cells / (kern_m * 1e-3) / 1e12
    out["roofline"] = {"bound": "alu", "achieved": achieved_tf, "peak": VALU_PEAK_TFLOPS,
                       "unit": "TFLOP/s", "frac": achieved_tf / VALU_PEAK_TFLOPS,
                       "traffic": measured_traffic(a.n), "kernel": "step_batch_kernel<2,float,0,0>",
                       # the FP32 rate with packed (two-wide) instructions, which the
                       # kernels do not use, for comparison
                       "peak_packed_fp32": 2 * VALU_PEAK_TFLOPS,
                       "frac_of_packed_fp32": achieved_tf / (2 * VALU_PEAK_TFLOPS),
                       "kernel_ms": kern_m, "flops_per_cell": flops}
    hbm = BYTES_PER_CELL["mixed"] * cells / (kern_m * 1e-3) / 1e9
    out["hbm_roofline"] = {"achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": hbm / HBM_PEAK_GBS, "bytes_per_cell": BYTES_PER_CELL["mixed"]}
    if not a.no_fp64:
        wall_d, kern_d = time_path(wl, pond.POND_FP64, a.steps, a.warmup)
        v64 = cells * a.steps / wall_d
        out["fp64"] = {"value": v64, "unit": "cell-updates/s", "ms_per_step": 1e3 * wall_d / a.steps,
                       "kernel_ms": kern_d,
                       "hbm_frac": BYTES_PER_CELL["fp64"] * cells / (kern_d * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "alu_frac": flops * cells / (kern_d * 1e-3) / 1e12 / VALU_PEAK_TFLOPS}
        out["mixed_over_fp64"] = value / v64
    if not a.no_multiscale:
        out["multiscale"] = multiscale_leg(max(1, a.steps // 2), a.warmup)
    if not a.no_walls:
        out["walls"] = walls_leg(a.n, max(1, a.steps // 2), a.warmup)
    if not a.no_force:
        out["force"] = force_leg(a.n, max(1, a.steps // 2), a.warmup)
    if not a.no_d2q25:
        out["d2q25"] = d2q25_leg(a.n, max(1, a.steps // 10), 2)
    if a.serving_requests > 0:
        sizes = tuple(int(v) for v in a.serving_sizes.split(","))
        out["serving"] = serving_leg(a.serving_requests, sizes, a.serving_arena_gb,
                                     a.serving_max_active)
    if a.copy_mb:
        x = torch.empty(a.copy_mb << 20, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
