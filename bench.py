"""Benchmark: cell-updates per second of the FP32 finite-volume step.

Workload (one GPU): shallow water on a 1024 x 1024 grid, FP32, reflective
walls, bed = 8 seeded Gaussians, free surface = 1 + 16 seeded Gaussian bumps,
zero velocity, HLLE flux, MINMOD reconstruction, Heun stages, CFL 0.4 with
the global wave-speed reduction every step.  A "step" is one full time step
(both stages and the Delta t reduction).  Inputs are resident in HBM before
the timed region.  Prints one JSON line.

Also measured (reported inside the line, not as `value`): the four-quadrant
Euler workload at 1024^2 (FP32, walls, 500 steps), a sample of the serving
stream (p50/p99 latency from arrival to completion) and the oracle on the host
cores over a bounded sample of the shallow-water workload.

The roofline object describes the stage kernel, which is bound by vector-ALU
issue: achieved = algorithmic FP32 operations per launch / mean launch time
(HIP events on the solver's stream over the timed steps), peak = the FP32
vector rate without packed math.  `traffic` is the measured HBM bytes per
launch from the committed counter summary, null once the kernel sources
differ from the ones the counters were taken on.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL_UPDATE = {"swe_bathy": 28, "euler": 32}  # read q (+b), write q, FP32
# Algorithmic FP32 operations of one cell-update of the shallow-water-over-a-
# bed step (MINMOD on h, hu, hv, eta; hydrostatic reconstruction; HLLE; bed
# source; Heun; CFL rate), counted from the formulas with an FMA as two
# operations: 114 per face and two faces per cell per stage, plus divergence,
# bed source and stage combine: 261 for stage 1, 270 for stage 2, and 12 for
# the CFL rate of the new state.
FLOP_PER_CELL_UPDATE = {"swe_bathy": 543, "euler": 715}
# Euler (HLLE, MINMOD on rho, rho u, rho v, E, Heun), counted the same way:
# per face 158 (reconstruction of 4 variables 36, pressure positivity checks
# of the two face states 18, HLLE with Roe-averaged speeds and enthalpy 104),
# two faces per cell and stage plus divergence and combine: 344 for stage 1,
# 356 for stage 2, and 15 for the CFL rate of the new state.
# FP32 vector peak without packed math: 256 CUs x 64 lanes x 2 (FMA) x 2.4 GHz.
ALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stage_kernel_swe_bathy_1024_fp32.json")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1000)
    p.add_argument("--warmup", type=int, default=100)
    p.add_argument("--n", type=int, default=1024, help="grid side")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-euler", action="store_true")
    p.add_argument("--learned-steps", type=int, default=1000,
                   help="64^2 learned steps timed for extra.learned_64_step_us (0: skip)")
    p.add_argument("--serving-requests", type=int, default=64,
                   help="requests in the serving sample (0: skip); p50/p99 at 0.8 of the saturated rate")
    p.add_argument("--cpu-seconds", type=float, default=12.0, help="target oracle CPU time for the baseline")
    p.add_argument("--calib-copy-mb", type=int, default=0,
                   help="before the run, copy this many MiB device-to-device once (a known-size kernel for "
                        "calibrating hardware traffic counters)")
    return p.parse_args()


def timed_run(solver, steps, warmup, torch):
    """Warm up, then time exactly `steps` steps with HIP events recorded on the
    solver's stream, bracketed by device synchronisation."""
    solver.run(warmup)
    torch.cuda.synchronize()
    st = solver.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    solver.run(steps)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3, wall


def measured_traffic():
    """Bytes per stage launch from the committed counter summary, or None
    when the kernel sources changed since the counters were taken."""
    from paper_2602_08670_amd import pmc_traffic

    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sources_sha256") != pmc_traffic.kernel_sources_sha256():
        return None
    return rec.get("bytes_per_launch")


def serving_sample(n_req):
    """The mixed SWE/Euler request stream (sizes 64..1024, 100..2000 steps)
    through the continuous-batching server: once with every request at t=0,
    then with Poisson arrivals at 0.8 of that saturated rate."""
    from paper_2602_08670_amd import serve_bench as sb

    stream = sb.request_stream(n_req, seed=0)
    ics = sb.ICCache()
    for kind, n, steps, sd in stream:
        ics.get(kind, n, sd)
    sat = sb.run_server_latency(stream, ics, np.zeros(n_req))
    rate = 0.8 * n_req / sat["wall_s"]
    poi = sb.run_server_latency(stream, ics, sb.arrivals(n_req, rate, 0))
    return {"requests": n_req, "saturated_mcups": round(sat["mcups"], 1), "poisson_rate_per_s": round(rate, 2),
            "p50_s": round(poi["p50_s"], 4), "p99_s": round(poi["p99_s"], 4), "poisson_mcups": round(poi["mcups"], 1)}


def learned_sample(steps, torch, direct=False, blend=False):
    """Latency of one learned (Heun) step on the 64^2 coarse grid of the
    learned-solver workload: periodic shallow water, fixed step = 32 x the
    2048^2 fine step, a network with seeded random weights (the step's cost
    does not depend on the weights).  HIP events on the solver's stream.
    direct: the direct face-state scheme's step instead; blend: the learned
    step with the flux-limiter blend of its face fluxes."""
    from paper_2602_08670_amd import fv, inputs
    from paper_2602_08670_amd import learned_solver as LS

    rng = np.random.default_rng(0)
    vec = (rng.standard_normal(49448) * 0.02).astype(np.float32)
    m = fv.Model(vec, fv.make_model_desc(mean=(1.0, 0.0, 0.0), inv_std=(10.0, 10.0, 10.0)))
    q0 = inputs.random_smooth_swe(64, seed=5).astype(np.float32)
    s = fv.Solver(q0, prec=fv.FV_F32, dt_fixed=LS.fine_dt(2048) * 32, learned=1)
    step = s.direct_step if direct else s.blend_step if blend else s.learned_step
    step(m, 20, want_stats=False)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    step(m, steps, want_stats=False)
    e1.record(s.stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / steps
    s.close()
    m.close()
    return round(us, 2)


def euler_learned_sample(steps, torch):
    """Latency of one learned Euler (Heun) step on the 64^2 coarse grid of the
    learned Euler workload: periodic Euler, fixed step = 8 x the 512^2 fine
    step, one solve, a network with seeded random weights.  HIP events on the
    network's stream."""
    from paper_2602_08670_amd import fv, inputs
    from paper_2602_08670_amd import learned_euler_solver as LE

    rng = np.random.default_rng(0)
    vec = (rng.standard_normal(fv.lib.fv_euler_net_param_count()) * 0.02).astype(np.float32)
    net = fv.EulerLearned(vec, 1, 64, 64, LE.fine_dt(512) * 8)
    q = torch.tensor(inputs.random_smooth_euler(64, seed=5)[None].astype(np.float32), device="cuda")
    net.step(q, 20)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(net.stream)
    net.step(q, steps)
    e1.record(net.stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / steps
    net.close()
    return round(us, 2)


def cpu_baseline(n, target_s, euler=False):
    """The oracle on the host cores over a bounded number of steps of the same
    workload (shallow water over the bed, or the Euler quadrants)."""
    import oracle
    from paper_2602_08670_amd import inputs

    threads = min(16, os.cpu_count() or 1)
    if euler:
        q0, b = inputs.euler_quadrants(n, seed=0), None
        cfg = oracle.Config(eqn=oracle.EULER, nx=n, ny=n, bc_x=oracle.WALL, bc_y=oracle.WALL, nthreads=threads)
        what = "Euler four-quadrant"
    else:
        q0, b = inputs.swe_bathy(n, seed=0)
        cfg = oracle.Config(nx=n, ny=n, bc_x=oracle.WALL, bc_y=oracle.WALL, nthreads=threads)
        what = "shallow-water bed"
    t0 = time.perf_counter()
    q1, *_ = oracle.run(cfg, q0, b, 1)
    one = time.perf_counter() - t0
    steps = max(1, min(200, int(target_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    oracle.run(cfg, q1, b, steps)
    el = time.perf_counter() - t0
    return {"value": round(n * n * steps / el / 1e6, 3), "unit": "Mcell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} steps of the {n}^2 FP64 {what} workload (after 1 untimed step), "
                      f"{el:.1f} s, OpenMP rows"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU domain "
              "decomposition is not implemented", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2602_08670_amd import fv, inputs

    n = args.n
    dev = torch.device("cuda:0")
    if args.calib_copy_mb:
        src = torch.ones(args.calib_copy_mb << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    q0, b = inputs.swe_bathy(n, seed=0)
    s = fv.Solver(q0, b, prec=fv.FV_F32, bc_x=fv.FV_BC_WALL, bc_y=fv.FV_BC_WALL, device=dev)
    gpu_s, wall_s = timed_run(s, args.steps, args.warmup, torch)
    t_sim, nsteps = s.time()
    s.close()
    cells = n * n * args.steps
    mcups = cells / gpu_s / 1e6
    launches = 2 * args.steps
    per_launch_s = gpu_s / launches
    # two stage launches per cell-update; per launch: half a cell-update per cell
    flop_per_launch = FLOP_PER_CELL_UPDATE["swe_bathy"] * n * n / 2
    achieved = flop_per_launch / per_launch_s / 1e12
    hbm_gbs = BYTES_PER_CELL_UPDATE["swe_bathy"] * n * n / 2 / per_launch_s / 1e9
    traffic = measured_traffic() if n == 1024 else None

    extra = {"wall_s": round(wall_s, 6), "sim_time": t_sim, "stage_launch_us": round(per_launch_s * 1e6, 3),
             "hbm_gbs_algorithmic": round(hbm_gbs, 1), "hbm_frac": round(hbm_gbs / HBM_PEAK_GBS, 4)}
    if not args.no_euler:
        qe = inputs.euler_quadrants(n, seed=0)
        se = fv.Solver(qe, prec=fv.FV_F32, bc_x=fv.FV_BC_WALL, bc_y=fv.FV_BC_WALL, device=dev)
        esteps = max(1, args.steps // 2)
        eg, _ = timed_run(se, esteps, max(1, args.warmup // 2), torch)
        se.close()
        e_launch = eg / (2 * esteps)
        e_ach = FLOP_PER_CELL_UPDATE["euler"] * n * n / 2 / e_launch / 1e12
        e_hbm = BYTES_PER_CELL_UPDATE["euler"] * n * n / 2 / e_launch / 1e9
        extra["euler"] = {
            "workload": f"euler_quadrants_{n}x{n}_fp32_walls_hlle_minmod_heun_cfl0.4", "steps": esteps,
            "value": round(n * n * esteps / eg / 1e6, 1), "unit": "Mcell-updates/s",
            "roofline": {"bound": "alu", "achieved": round(e_ach, 2), "peak": round(ALU_PEAK_TFLOPS, 1),
                         "unit": "TFLOP/s", "frac": round(e_ach / ALU_PEAK_TFLOPS, 4), "traffic": None},
            "hbm_gbs_algorithmic": round(e_hbm, 1), "hbm_frac": round(e_hbm / HBM_PEAK_GBS, 4)}
        if not args.no_cpu_baseline:
            extra["euler"]["cpu_baseline"] = cpu_baseline(n, args.cpu_seconds / 3, euler=True)

    if args.learned_steps > 0:
        extra["learned_64_step_us"] = learned_sample(args.learned_steps, torch)
        extra["direct_64_step_us"] = learned_sample(args.learned_steps, torch, direct=True)
        extra["blend_64_step_us"] = learned_sample(args.learned_steps, torch, blend=True)
        extra["euler_learned_64_step_us"] = euler_learned_sample(args.learned_steps, torch)

    if args.serving_requests > 0:
        extra["serving"] = serving_sample(args.serving_requests)

    line = {
        "metric": "Mcell-updates/s FP32 SWE 1024^2 + % HBM roofline; p50/p99 solve latency",
        "value": round(mcups, 1),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(gpu_s / args.steps * 1e3, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Gaussian bed and surface bumps)",
        "config": {"workload": f"swe_bathy_{n}x{n}_fp32_walls_hlle_minmod_heun_cfl0.4", "nx": n, "ny": n,
                   "steps": args.steps, "parallelism": "single-gpu"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": round(ALU_PEAK_TFLOPS, 1),
                     "unit": "TFLOP/s", "frac": round(achieved / ALU_PEAK_TFLOPS, 4), "traffic": traffic},
        "extra": extra,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(n, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
