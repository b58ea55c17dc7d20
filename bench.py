#!/usr/bin/env python3
"""Benchmark of the ideal-MHD step on one MI355X.

Workload: 3D decaying MHD turbulence, 256^3 periodic, FP64, PLM van Leer +
HLLD + upwind CT + SSP-RK2, CFL 0.3, seeded synthetic initial data (rms Mach
1, B0 = 0.1 along x plus a divergence-free perturbation). One "step" is the
whole hot path: the CFL time step on the device, then both RK stages
(primitive recovery, reconstruction, Riemann solve, EMF, update). The state
is resident in HBM before the timed region; dt never leaves the device.

Prints one JSON line: Mcell-updates/s, the HBM-roofline fraction of the step
(320 algorithmic bytes per cell-update), the dominant kernel's roofline entry
measured with HIP events inside the timed region, and the CPU oracle timed on
a bounded sample of the same workload on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # B/s, MI355X HBM3E
FP64_PEAK = 78.6e12        # flop/s, MI355X FP64 vector
STEP_BYTES = 320           # algorithmic HBM bytes per cell-update of a fused RK2 step
METRIC = ("Mcell-updates/s at 256³ (FP64 vs mixed FP32/FP64) + % HBM roofline; "
          "adjoint step/s")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes_per_cell(name: str, dim: int) -> float:
    """Algorithmic HBM bytes per cell of one launch of each kernel, from what
    the kernel must read and write once (halo re-reads excluded)."""
    faces_out = dim * (5 if dim == 3 else 6) + dim * 4    # fluxes + alpha+- + 2 velocities
    table = {
        "faces": 8 * (8 + faces_out),                       # read U, write face records
        "emf": 8 * (dim * 4 + dim + (3 if dim == 3 else 1)),  # read alpha,v, b; write E
        "update": 8 * (faces_out - dim * 4 + (3 if dim == 3 else 1) + 8 + 8),  # fluxes, E, U, out
        "cfl": 8 * 8,
    }
    return float(table.get(name, 0.0))


def time_gpu(setup, U0, steps, warmup, timing=True):
    import torch
    from paper_2511_20337_amd import mhd
    dev = torch.device("cuda:0")
    ctx = mhd.Context(setup, dev)
    U = torch.from_numpy(U0).to(dev)
    for _ in range(warmup):
        ctx.dt_device(U)
        ctx.step_device_dt(U)
    torch.cuda.synchronize()
    if timing:
        mhd.mhd_timing(ctx.ctx, True)
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.dt_device(U)
        ctx.step_device_dt(U)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = mhd.mhd_timing_read(ctx.ctx) if timing else {}
    if timing:
        mhd.mhd_timing(ctx.ctx, False)
    ctx.check()
    return elapsed, kt, U


def cpu_baseline(n_sample: int, setup_fn):
    """The oracle, untuned, on the same generator at n_sample^3: one dt + one
    RK2 step with every host thread this process may use."""
    import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    setup, U = setup_fn(n_sample)
    c = O.cfg_from(setup, nthreads=threads)
    t0 = time.perf_counter()
    dt = O.dt(c, U)
    O.step(c, U, dt)
    el = time.perf_counter() - t0
    cells = n_sample ** 3
    return {"value": cells / el / 1e6, "unit": "Mcell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "same turbulence generator at %d^3, 1 CFL dt + 1 RK2 step (%.1f s), "
                      "%d OpenMP threads" % (n_sample, el, threads)}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256, help="grid cells per side")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-n", type=int, default=128, help="oracle sample size per side")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    from paper_2511_20337_amd import workloads as W

    def make(n):
        return W.turbulence_3d(n)

    log("generating 3D turbulence %d^3" % args.n)
    setup, U0 = make(args.n)
    ncell = args.n ** 3
    log("timing %d steps after %d warmup" % (args.steps, args.warmup))
    elapsed, kt, _ = time_gpu(setup, U0, args.steps, args.warmup)
    value = ncell * args.steps / elapsed / 1e6
    ms_per_step = elapsed / args.steps * 1e3

    # dominant kernel by total event time
    dom = max(kt.items(), key=lambda kv: kv[1][0])
    name, (tot_ms, launches) = dom
    avg_s = tot_ms / launches / 1e3
    bpc = kernel_bytes_per_cell(name, 3)
    achieved = bpc * ncell / avg_s
    roofline = {"kernel": name, "bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": achieved / HBM_PEAK, "traffic": None,
                "avg_launch_ms": avg_s * 1e3, "bytes_per_cell": bpc}
    kernels = {k: {"avg_ms": v[0] / v[1], "launches": v[1], "share": v[0] / sum(x[0] for x in kt.values())}
               for k, v in kt.items() if v[1]}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "turbulence_3d_%d" % args.n, "grid": [args.n] * 3,
                   "limiter": "vanleer", "riemann": "hlld", "emf": "uct_hll",
                   "integrator": "ssp_rk2", "cfl": 0.3, "precision": "fp64"},
        "hbm_roofline_frac_step": value * 1e6 * STEP_BYTES / HBM_PEAK,
        "roofline": roofline,
        "kernels": kernels,
    }
    if not args.no_cpu:
        log("cpu baseline: oracle at %d^3" % args.cpu_n)
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, make)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
