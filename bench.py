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


_T0 = time.perf_counter()


def log(*a):
    """Progress line on stderr, prefixed with the seconds since start."""
    print("[%6.1f s]" % (time.perf_counter() - _T0), *a, file=sys.stderr, flush=True)


# Roofline of the dominant kernel, the face kernel (reconstruction + Riemann
# solve of every lower face, with primitive recovery), per cell:
#  flops: operations of the method's definition in those phases (add/sub, mul,
#         div, sqrt one each), counted by oracle/count_flops.py on the initial
#         state of this workload at 256^3 (3D turbulence, van Leer, HLLD);
#  bytes: the state it must read once, 64 B; the face records it writes are an
#         artefact of splitting the stage into kernels, not algorithmic traffic.
# The kernel's roof is the slower of the two: flops at the vector peak of the
# arithmetic's precision (FP64 78.6 TFLOP/s; FP32 157.3 in the mixed mode) or
# bytes at 8 TB/s; frac = that time / the measured time per launch.
FACE_FLOPS = 1343.8
FACE_BYTES = 64
FP32_PEAK = 157.3e12
# HBM bytes per cell of one face-kernel launch, rocprofv3 FETCH_SIZE x 2.0 and
# WRITE_SIZE x 1.0 (the copy-kernel calibration), for the kernel as it stands.
FACE_TRAFFIC = {"fp64": 189.0 + 216.0, "mixed": 190.0 + 108.0}
# HBM bytes per cell of one whole step, the same counters summed over its
# launches (two of faces and EMF, the updates of both stages): what the
# three-kernel stage moves beside the 320 algorithmic bytes.
STEP_TRAFFIC = {"fp64": 1984.7, "mixed": 1320.4}
# WENO-Z face kernel on the 3D Orszag-Tang problem (FP64, HLLD): algorithmic
# flops per cell of the oracle's face phase on that workload at 256^3 (count_flops.py;
# its textbook WENO-Z with seven divisions per value, each one flop), and the
# HBM bytes per cell counted at 352^3 (reads past L2 x2.0, writes x1.0).
WENO_FACE_FLOPS = 4039.4
WENO_FACE_TRAFFIC = 339.8 + 240.0


def face_roofline(kt, ncell, precision="fp64"):
    """Roofline entry of the face kernel from its HIP-event times."""
    tot_ms, launches = kt["faces"]
    avg_s = tot_ms / launches / 1e3
    fpeak = FP64_PEAK if precision == "fp64" else FP32_PEAK
    t_alu = FACE_FLOPS * ncell / fpeak
    t_hbm = FACE_BYTES * ncell / HBM_PEAK
    traffic = FACE_TRAFFIC[precision] * ncell
    out = {"kernel": "faces", "avg_launch_ms": avg_s * 1e3, "flops_per_cell": FACE_FLOPS,
           "bytes_per_cell": FACE_BYTES, "traffic": traffic, "traffic_unit": "bytes per launch",
           "hbm_counted_GBps": traffic / avg_s / 1e9,
           "alu_frac": t_alu / avg_s, "hbm_frac": t_hbm / avg_s}
    if t_alu >= t_hbm:
        out.update({"bound": "alu", "achieved": FACE_FLOPS * ncell / avg_s / 1e12,
                    "peak": fpeak / 1e12, "unit": "TFLOP/s", "frac": t_alu / avg_s})
    else:
        out.update({"bound": "hbm", "achieved": FACE_BYTES * ncell / avg_s / 1e9,
                    "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": t_hbm / avg_s})
    return out


def time_gpu(setup, U0, steps, warmup, timing=True):
    """Time `steps` whole steps (CFL dt on the device + RK2 step, one
    mhd_step_cfl call each) after `warmup` steps.
    Returns (seconds, per-kernel event totals, final state, physical?)."""
    import torch
    from paper_2511_20337_amd import mhd
    dev = torch.device("cuda:0")
    ctx = mhd.Context(setup, dev)
    U = torch.from_numpy(U0).to(dev)
    for _ in range(warmup):
        ctx.step_cfl(U)
    torch.cuda.synchronize()
    if timing:
        mhd.mhd_timing(ctx.ctx, True)
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.step_cfl(U)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = mhd.mhd_timing_read(ctx.ctx) if timing else {}
    if timing:
        mhd.mhd_timing(ctx.ctx, False)
    try:
        ctx.check()
        physical = True
    except mhd.Unphysical:
        physical = False
    return elapsed, kt, U, physical


def time_adjoint(n, nsteps, every):
    """Kelvin-Helmholtz n^2: N forward steps with checkpoints, then the
    checkpointed backward (segment replay + adjoint steps). Returns adjoint
    steps/s of the backward pass and the forward steps/s."""
    import torch
    from paper_2511_20337_amd import adjoint as AD, mhd, workloads as W
    dev = torch.device("cuda:0")
    s, U, _ = W.kelvin_helmholtz_2d(n)
    ctx = mhd.Context(s, dev, with_adjoint=True)
    U0 = torch.from_numpy(U).to(dev)
    dts, _ = AD.record_dts(ctx, U0, nsteps)
    return _time_backward(AD, ctx, U0, dts, every)


def _time_backward(AD, ctx, U0, dts, every):
    """Forward with checkpoints, then the checkpointed backward, after an
    untimed two-step warmup of both (first launches load the kernels).
    Returns (adjoint steps/s, forward steps/s)."""
    import torch
    w = U0.clone().requires_grad_(True)
    AD.run_with_grad(ctx, w, dts[:2], every=every).backward(torch.ones_like(U0))
    x = U0.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = AD.run_with_grad(ctx, x, dts, every=every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out.backward(torch.ones_like(out))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    n = len(dts)
    return n / (t2 - t1), n / (t1 - t0)


# Checkpoint interval of the adjoint measurements at 512^2 and 256^3: every
# state of the forward pass is kept (64 x 16.8 MB, 16 x 1.07 GB), so the
# backward replays nothing; HBM holds them easily next to the workspaces.
ADJ_EVERY = 1

# The largest cube on which the blast's checkpointed 16-step adjoint fits in one
# MI355X's 288 GB: the library's forward and adjoint workspaces (188 doubles per
# cell with SSP-RK2) plus the state, four checkpoints, the replayed segment and
# the two cotangents (about 96 more) make 284 doubles per cell, 204 GB at 448^3
# (305 GB at 512^3; the 640^3 of the blast configuration would need 596 GB).
ADJ_LARGE_N = 448


def time_adjoint_blast(n, nsteps, every, integrator="rk2"):
    """Magnetised blast n^3 in FP64: N forward steps with checkpoints, then the
    checkpointed backward. Returns adjoint steps/s and forward steps/s."""
    import torch
    from paper_2511_20337_amd import adjoint as AD, mhd, workloads as W
    dev = torch.device("cuda:0")
    s, U = W.blast_3d(n, precision="fp64")
    s = dict(s, integrator=integrator)
    ctx = mhd.Context(s, dev, with_adjoint=True)
    U0 = torch.from_numpy(U).to(dev)
    del U
    dts, _ = AD.record_dts(ctx, U0, nsteps)
    return _time_backward(AD, ctx, U0, dts, every)


def time_2d_graph(n=128, steps=100, per_graph=10):
    """The 2D Orszag-Tang configuration, 128^2: microseconds per step run
    eagerly (one library call per step, each some ten kernel launches on
    16 K cells: launch-bound) and with per_graph steps captured in a HIP graph
    (torch.cuda.CUDAGraph) that is replayed."""
    import torch
    from paper_2511_20337_amd import mhd, workloads as W
    dev = torch.device("cuda:0")
    s, U0 = W.orszag_tang_2d(n)
    ctx = mhd.Context(s, dev)
    U = torch.from_numpy(U0).to(dev)
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    for _ in range(5):
        ctx.step_cfl(U, dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.step_cfl(U, dt)
    torch.cuda.synchronize()
    eager = (time.perf_counter() - t0) / steps
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(per_graph):
            ctx.step_cfl(U, dt)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps // per_graph):
        g.replay()
    torch.cuda.synchronize()
    graph = (time.perf_counter() - t0) / (steps // per_graph * per_graph)
    return {"workload": "orszag_tang_2d_%d" % n, "us_per_step_eager": eager * 1e6,
            "us_per_step_graph": graph * 1e6, "steps": steps, "steps_per_graph": per_graph}


def cpu_baseline(n_sample: int, setup_fn, steps: int = 2):
    """The oracle, untuned, on the same generator at n_sample^3: `steps` steps
    (CFL dt + RK2 step each) with every host thread this process may use."""
    import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    setup, U = setup_fn(n_sample)
    c = O.cfg_from(setup, nthreads=threads)
    t0 = time.perf_counter()
    O.run(c, U, steps)
    el = time.perf_counter() - t0
    cells = n_sample ** 3
    return {"value": cells * steps / el / 1e6, "unit": "Mcell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "same turbulence generator at %d^3, %d steps of CFL dt + RK2 step "
                      "(%.1f s), %d OpenMP threads" % (n_sample, steps, el, threads)}


def copy_probe(mib: int) -> int:
    """A plain copy of known size, timed, as the reference for HBM counters;
    then the practical HBM rates of a copy, a read-only sum and a fill of the
    same buffers (HIP events over ten calls each, after three untimed)."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / 5
    rates = {}
    for name, fn, nbytes in (("copy", lambda: dst.copy_(src), 2 * n * 8),
                             ("sum", lambda: src.sum(), n * 8),
                             ("fill", lambda: dst.fill_(1.0), n * 8)):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            fn()
        e1.record()
        torch.cuda.synchronize()
        rates[name] = nbytes / (e0.elapsed_time(e1) / 10 * 1e-3) / 1e9
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8,
                      "copies": 5, "GBps": 2 * n * 8 / el / 1e9,
                      "event_GBps": rates}), flush=True)
    return 0


def weno_roofline(kt, ncell):
    """ALU roofline entry of the WENO-Z face kernel from its event times."""
    tot_ms, launches = kt["faces"]
    avg_s = tot_ms / launches / 1e3
    achieved = WENO_FACE_FLOPS * ncell / avg_s
    return {"kernel": "faces", "bound": "alu", "achieved": achieved / 1e12,
            "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK,
            "traffic": WENO_FACE_TRAFFIC * ncell, "traffic_unit": "bytes per launch",
            "avg_launch_ms": avg_s * 1e3, "flops_per_cell": WENO_FACE_FLOPS}


def only_part(part, n, steps, warmup):
    """One extra measurement alone, printed as one JSON line."""
    from paper_2511_20337_amd import workloads as W
    if part == "mixed":
        sm, Um = W.turbulence_3d_lowbeta(n)
        el, kt, _, phys = time_gpu(sm, Um, steps, warmup)
        out = {"part": part, "value": n ** 3 * steps / el / 1e6, "unit": "Mcell-updates/s",
               "workload": "turbulence_3d_lowbeta_%d" % n, "physical": phys,
               "kernels": {k: {"avg_ms": v[0] / v[1]} for k, v in kt.items() if v[1]}}
    elif part == "ot3d_wenoz":
        so, Uo = W.orszag_tang_3d(n, limiter="wenoz")
        el, kt, _, phys = time_gpu(dict(so, integrator="rk3", emf="uct_hlld"), Uo, steps, warmup)
        out = {"part": part, "value": n ** 3 * steps / el / 1e6, "unit": "Mcell-updates/s",
               "workload": "orszag_tang_3d_%d wenoz ssp_rk3 hlld uct_hlld" % n, "physical": phys,
               "ms_per_step": el / steps * 1e3,
               "kernels": {k: {"avg_ms": v[0] / v[1]} for k, v in kt.items() if v[1]},
               "roofline": weno_roofline(kt, n ** 3)}
    elif part == "glm":
        sg, Ug = W.glm_from_ct(*W.turbulence_3d(n))
        el, kt, _, phys = time_gpu(sg, Ug, steps, warmup)
        out = {"part": part, "value": n ** 3 * steps / el / 1e6, "unit": "Mcell-updates/s",
               "workload": "turbulence_3d_%d glm" % n, "physical": phys,
               "ms_per_step": el / steps * 1e3,
               "kernels": {k: {"avg_ms": v[0] / v[1]} for k, v in kt.items() if v[1]}}
    elif part == "ot2d_graph":
        out = dict({"part": part}, **time_2d_graph())
    elif part == "adjoint":
        adj, fwd = time_adjoint(512, 64, ADJ_EVERY)
        out = {"part": part, "value": adj, "unit": "adjoint steps/s", "forward_steps_per_s": fwd,
               "workload": "kelvin_helmholtz_2d_512"}
    elif part == "adjoint_3d_large":
        adj, fwd = time_adjoint_blast(ADJ_LARGE_N, 16, 4)
        out = {"part": part, "value": adj, "unit": "adjoint steps/s", "forward_steps_per_s": fwd,
               "workload": "blast_3d_%d_fp64 ssp_rk2" % ADJ_LARGE_N}
    else:
        integ = "rk3" if part == "adjoint_3d_rk3" else "rk2"
        adj, fwd = time_adjoint_blast(256, 16, ADJ_EVERY, integ)
        out = {"part": part, "value": adj, "unit": "adjoint steps/s", "forward_steps_per_s": fwd,
               "workload": "blast_3d_256_fp64 ssp_%s" % integ}
    print(json.dumps(out), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256, help="grid cells per side")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-n", type=int, default=256, help="oracle sample size per side")
    ap.add_argument("--cpu-steps", type=int, default=2, help="oracle sample steps")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the mixed-precision and adjoint measurements")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (calibrates the "
                         "HBM byte counters) and exit")
    ap.add_argument("--only", choices=("mixed", "ot3d_wenoz", "glm", "ot2d_graph", "adjoint",
                                       "adjoint_3d", "adjoint_3d_rk3", "adjoint_3d_large"),
                    default=None,
                    help="run only this extra measurement and print it (for profiling)")
    args = ap.parse_args(argv)
    if args.copy_probe:
        return copy_probe(args.copy_probe)
    if args.only:
        return only_part(args.only, args.n, args.steps, args.warmup)
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    from paper_2511_20337_amd import workloads as W

    def make(n):
        return W.turbulence_3d(n)

    log("generating 3D turbulence %d^3" % args.n)
    setup, U0 = make(args.n)
    ncell = args.n ** 3
    log("timing %d steps after %d warmup" % (args.steps, args.warmup))
    elapsed, kt, _, physical = time_gpu(setup, U0, args.steps, args.warmup)
    value = ncell * args.steps / elapsed / 1e6
    ms_per_step = elapsed / args.steps * 1e3

    roofline = face_roofline(kt, ncell)
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
        "step_bytes_per_cell": {"algorithmic": STEP_BYTES, "counted": STEP_TRAFFIC["fp64"]},
        "physical": physical,
        "roofline": roofline,
        "kernels": kernels,
    }
    if not args.no_extras:
        del U0
        log("mixed precision: low-beta turbulence %d^3" % args.n)
        sm, Um = W.turbulence_3d_lowbeta(args.n)
        el_m, kt_m, _, phys_m = time_gpu(sm, Um, args.steps, args.warmup)
        del Um
        vm = ncell * args.steps / el_m / 1e6
        out["mixed"] = {"value": vm, "unit": "Mcell-updates/s", "ms_per_step": el_m / args.steps * 1e3,
                        "hbm_roofline_frac_step": vm * 1e6 * STEP_BYTES / HBM_PEAK,
                        "step_bytes_per_cell": {"algorithmic": STEP_BYTES,
                                                "counted": STEP_TRAFFIC["mixed"]},
                        "roofline": face_roofline(kt_m, ncell, "mixed"),
                        "physical": phys_m,
                        "config": {"workload": "turbulence_3d_lowbeta_%d" % args.n, "mach": 3,
                                   "beta": 0.01, "precision": "mixed"},
                        "kernels": {k: {"avg_ms": v[0] / v[1]} for k, v in kt_m.items() if v[1]}}
        out["large"] = {}
        # the step counts these workloads are named with (C3: 50 steps at 384^3;
        # C5: 100 steps of the blast at 640^3)
        for name, fn, n, steps_l in (("turbulence_3d_lowbeta_384", W.turbulence_3d_lowbeta, 384, 50),
                                     ("blast_3d_640", W.blast_3d, 640, 100)):
            log("mixed precision, large grid: %s, %d steps" % (name, steps_l))
            sl, Ul = fn(n)
            el_l, kt_l, _, phys_l = time_gpu(sl, Ul, steps_l, 1)
            del Ul
            vl = n ** 3 * steps_l / el_l / 1e6
            out["large"][name] = {"value": vl, "unit": "Mcell-updates/s", "steps": steps_l,
                                  "ms_per_step": el_l / steps_l * 1e3, "physical": phys_l,
                                  "precision": sl["precision"], "limiter": sl["limiter"],
                                  "kernels": {k: {"avg_ms": v[0] / v[1]} for k, v in kt_l.items()
                                              if v[1]}}
        log("the paper's 3D Orszag-Tang problem at 352^3 (its per-GPU size), FP64")
        so, Uo = W.orszag_tang_3d(352)
        steps_o = max(1, args.steps // 5)
        el_o, kt_o, _, phys_o = time_gpu(so, Uo, steps_o, 1)
        del Uo
        out["orszag_tang_3d"] = {
            "value": 352 ** 3 * steps_o / el_o / 1e6, "unit": "Mcell-updates/s", "steps": steps_o,
            "ms_per_step": el_o / steps_o * 1e3, "physical": phys_o,
            "config": {"workload": "orszag_tang_3d_352", "precision": "fp64", "limiter": "vanleer",
                       "riemann": "hlld", "integrator": "ssp_rk2"},
            "kernels": {k: {"avg_ms": v[0] / v[1]} for k, v in kt_o.items() if v[1]},
            "paper_context": {"value": 37.8, "unit": "Mcell-updates/s per GPU",
                              "hardware": "NVIDIA H100 (4 per node)",
                              "scheme": "WENO-Z + RK3 + HLLD + CT (UCT-HLLD), FP64",
                              "note": "context only: another scheme on other hardware"}}
        log("the same with SSP-RK3, the paper's integrator")
        so3, Uo3 = W.orszag_tang_3d(352)
        so3 = dict(so3, integrator="rk3")
        el_o3, kt_o3, _, phys_o3 = time_gpu(so3, Uo3, steps_o, 1)
        del Uo3
        out["orszag_tang_3d"]["rk3"] = {
            "value": 352 ** 3 * steps_o / el_o3 / 1e6, "unit": "Mcell-updates/s",
            "ms_per_step": el_o3 / steps_o * 1e3, "physical": phys_o3,
            "kernels": {k: {"avg_ms": v[0] / v[1]} for k, v in kt_o3.items() if v[1]}}
        log("the same with the paper's scheme: WENO-Z + SSP-RK3 + HLLD + CT (UCT-HLLD)")
        sow, Uow = W.orszag_tang_3d(352, limiter="wenoz")
        sow = dict(sow, integrator="rk3", emf="uct_hlld")
        el_ow, kt_ow, _, phys_ow = time_gpu(sow, Uow, steps_o, 1)
        del Uow
        out["orszag_tang_3d"]["wenoz_rk3"] = {
            "value": 352 ** 3 * steps_o / el_ow / 1e6, "unit": "Mcell-updates/s",
            "ms_per_step": el_ow / steps_o * 1e3, "physical": phys_ow,
            "kernels": {k: {"avg_ms": v[0] / v[1]} for k, v in kt_ow.items() if v[1]},
            "roofline": weno_roofline(kt_ow, 352 ** 3)}
        log("GLM divergence cleaning: the same turbulence %d^3 on nine cell-centred fields" % args.n)
        sg, Ug = W.glm_from_ct(*W.turbulence_3d(args.n))
        steps_g = max(1, args.steps // 5)
        el_g, kt_g, _, phys_g = time_gpu(sg, Ug, steps_g, 1)
        del Ug
        out["glm"] = {"value": ncell * steps_g / el_g / 1e6, "unit": "Mcell-updates/s",
                      "steps": steps_g, "ms_per_step": el_g / steps_g * 1e3, "physical": phys_g,
                      "config": {"workload": "turbulence_3d_%d" % args.n, "divb": "glm",
                                 "limiter": "vanleer", "riemann": "hlld", "integrator": "ssp_rk2"},
                      "kernels": {k: {"avg_ms": v[0] / v[1]} for k, v in kt_g.items() if v[1]}}
        log("2D Orszag-Tang 128^2: eager steps and steps replayed from a HIP graph")
        out["orszag_tang_2d"] = time_2d_graph()
        log("adjoint: Kelvin-Helmholtz 512^2, 64 steps, every state kept")
        adj, fwd = time_adjoint(512, 64, ADJ_EVERY)
        out["adjoint"] = {"value": adj, "unit": "adjoint steps/s", "forward_steps_per_s": fwd,
                          "config": {"workload": "kelvin_helmholtz_2d_512", "steps": 64,
                                     "checkpoint_every": ADJ_EVERY}}
        log("adjoint: blast 256^3 FP64, 16 steps, every state kept")
        adj3, fwd3 = time_adjoint_blast(256, 16, ADJ_EVERY)
        out["adjoint_3d"] = {"value": adj3, "unit": "adjoint steps/s",
                             "forward_steps_per_s": fwd3,
                             "config": {"workload": "blast_3d_256_fp64", "steps": 16,
                                        "checkpoint_every": ADJ_EVERY}}
        log("adjoint: the same with checkpoints every 4 steps (segments replayed)")
        adj34, fwd34 = time_adjoint_blast(256, 16, 4)
        out["adjoint_3d"]["checkpoint_every_4"] = {"value": adj34, "unit": "adjoint steps/s",
                                                   "forward_steps_per_s": fwd34}
        log("adjoint: the same with SSP-RK3")
        adj3r, fwd3r = time_adjoint_blast(256, 16, ADJ_EVERY, "rk3")
        out["adjoint_3d"]["rk3"] = {"value": adj3r, "unit": "adjoint steps/s",
                                    "forward_steps_per_s": fwd3r}
        log("adjoint: blast %d^3 FP64, the largest cube whose adjoint fits in HBM" % ADJ_LARGE_N)
        import torch
        torch.cuda.empty_cache()
        adjl, fwdl = time_adjoint_blast(ADJ_LARGE_N, 16, 4)
        out["adjoint_3d"]["large"] = {"value": adjl, "unit": "adjoint steps/s",
                                      "forward_steps_per_s": fwdl,
                                      "workload": "blast_3d_%d_fp64" % ADJ_LARGE_N,
                                      "checkpoint_every": 4}
    if not args.no_cpu:
        log("cpu baseline: oracle at %d^3" % args.cpu_n)
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, make, args.cpu_steps)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
